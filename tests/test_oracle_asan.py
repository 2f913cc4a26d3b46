"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): its C code, built with -fsanitize=address,undefined, runs every
entry point on small cases in a child process that preloads the ASan
runtime; any out-of-bounds access, use after free or undefined behaviour
ends that process with a report, which fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
from oracle import oracle as O
from paper_1410_0260_amd import synth

X = synth.mixture_points(700, 6, 3, 3, 1e-3, 5)
W = synth.weights(700, 2, 6)
for p in (O.Params(m=32, kappa=8, smax=16, ell=36, tau=1e-6, h=0.7, seed=3),
          O.Params(m=40, kappa=6, smax=12, ell=30, tau=1e-5, h=0.0, bw_neighbor=4, seed=4),
          O.Params(m=24, kappa=5, smax=10, ell=30, tau=0.0, h=0.5, seed=5, prune_levels=2)):
    st = O.run_askit(X, W, p, record=True)
    Y = synth.mixture_points(60, 6, 3, 3, 1e-3, 7, basis_seed=5)
    O.query(dict(st, W=W, Wsk=O.upward(st["nodes"], W[st["perm"]].astype(np.float64), st["sk"], p.smax)), Y)
ki, kd = O.rpknn(X, 8, 40, 3, 11)
st = O.run_askit(X, W, O.Params(m=32, kappa=8, smax=16, ell=36, tau=1e-6, h=0.7, seed=3), knn_lists=(ki, kd))
nodes, perm = O.tree(X, 32)
iperm = np.empty(len(X), np.int32)
iperm[perm] = np.arange(len(X), dtype=np.int32)
O.prune_visits(X, perm, nodes, np.concatenate([iperm[:, None], iperm[ki]], axis=1))
O.direct(X[:50], X, W, 0.7)
maps = open("/proc/self/maps").read()
assert "liboracle_asan.so" in maps and "libasan" in maps, "the sanitizer build was not the one loaded"
print("sanitized oracle run: ok")
'''


def _runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_sanitizers():
    rt = _runtime()
    if rt is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    from oracle import build
    build.build_asan(force=False)
    env = dict(os.environ, ASKIT_ORACLE_ASAN="1", LD_PRELOAD=rt, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    report = r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert r.returncode == 0, report
    assert "sanitized oracle run: ok" in r.stdout
