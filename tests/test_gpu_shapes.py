"""Parity at the shapes of the mixed-precision and batched workloads (needs an
MI355X), on sizes the FP64 oracle finishes in about a minute:

  * 1000-dimensional points (6-dim intrinsic, 8 components, noise variance
    1e-4), m = 512, kappa = 32, s <= 256, l = 276, 16 right-hand sides, on a
    2^14-point slice of that workload's generator, in the FP32 form and in the
    bf16 hi/lo precision form;
  * a batch of uneven instances shaped like the batched workload -- one of
    65,536 points in 64-D, others of 20,000 and 3,001 points in 32-D and 16-D --
    with m = 256, kappa = 16, s <= 128, l = 148 and the variable bandwidth
    h_j = distance to the 16th neighbour.

Neighbour lists, tree and skeletons must match bit for bit; u within 1e-5
relative L2 of the oracle's u in FP32 (1e-4 in the bf16 form), per RHS, at
seeded sampled targets."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth
from tests.gpu_common import rel
from tests.test_gpu_parity import gparams

pytestmark = pytest.mark.gpu


def _oracle_u_at(st, X, W, p, tg):
    Wsk = O.upward(st["nodes"], W[st["perm"]].astype(np.float64), st["sk"], p.smax)
    nb = O.self_neighbours(st, tg)
    return O.evaluate(X[tg], nb, X, st["perm"], st["nodes"], st["hsrc"], p.h, W, st["sk"], Wsk, p.smax,
                      record=False).U


def _compare_structures(st, g, rows):
    assert np.array_equal(g["perm"], st["perm"])
    assert np.array_equal(g["knn_idx"][rows], st["knn_idx"][rows])
    assert np.array_equal(g["knn_d"][rows], st["knn_d"][rows])
    sk = st["sk"]
    for a in range(1, len(st["nodes"])):
        k = sk.k[a]
        same = g["k"][a] == k and np.array_equal(g["S"][a, :k], sk.S[a, :k])
        assert same or min(sk.piv_margin[a], sk.rank_margin[a]) < 1e-10, f"node {a}"
        assert same, f"certified near-tie at node {a} (none expected)"


@pytest.fixture(scope="module")
def wide():
    wl = synth.mixed_1000d()
    N = 1 << 14
    X = synth.mixture_points(N, wl.d, wl.q, wl.n_comp, wl.noise_var, wl.seed, wl.spread)
    W = synth.weights(N, wl.R, wl.seed)
    p = O.Params.from_workload(wl)
    print(f"\n[shape 1000-D] oracle setup, N={N}", flush=True)
    st = O.setup(X, p)
    tg = np.sort(np.random.default_rng(31).choice(N, 1200, replace=False))
    print("[shape 1000-D] oracle evaluation at 1200 targets", flush=True)
    Uo = _oracle_u_at(st, X, W, p, tg)
    return X, W, p, st, tg, Uo


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_1000d_slice(wide, precision):
    import torch
    from paper_1410_0260_amd import askit as A
    X, W, p, st, tg, Uo = wide
    prec = A.PREC_BF16X3 if precision == "bf16x3" else A.PREC_FP32
    h = A.setup(torch.from_numpy(X).cuda(), gparams(p, precision=prec))
    h.update_weights(torch.from_numpy(W).cuda())
    U = h.evaluate().cpu().numpy().astype(np.float64)
    g = h.structures()
    h.close()
    print(f"[shape 1000-D {precision}] rows certified by the approximate pass: "
          f"{len(X) - g['info']['knn_uncertified_rows']} of {len(X)}", flush=True)
    _compare_structures(st, g, np.arange(len(X)))
    tol = 1e-4 if precision == "bf16x3" else 1e-5
    errs = [rel(U[tg, r], Uo[:, r]) for r in range(W.shape[1])]
    print(f"[shape 1000-D {precision}] relative L2 error per RHS: max {max(errs):.2e}", flush=True)
    assert max(errs) < tol


BATCH_SHAPES = [(65536, 64), (20000, 32), (3001, 16)]


def test_batched_shape_matches_oracle():
    import torch
    from paper_1410_0260_amd import askit as A
    base = synth.batched_instances(1)[0]
    p = O.Params(m=base.m, kappa=base.kappa, smax=base.smax, ell=base.ell_eff, tau=base.tau, h=0.0,
                 bw_neighbor=base.bw_neighbor, seed=base.seed)
    Xs = [synth.mixture_points(n, d, 4, 1, 1e-3, 7000 + i) for i, (n, d) in enumerate(BATCH_SHAPES)]
    b = A.Batch([torch.from_numpy(X).cuda() for X in Xs], gparams(p))
    W = synth.weights(b.rows, 2, 4321)
    Ub = b.run(torch.from_numpy(W).cuda(), torch.empty((b.rows, 2), device="cuda")).cpu().numpy()
    gs = [b.instance(i).structures() for i in range(len(Xs))]
    b.close()
    for i, X in enumerate(Xs):
        N = len(X)
        print(f"[shape batched] instance {i}: N={N} d={X.shape[1]}, oracle setup", flush=True)
        st = O.setup(X, p)
        Wi = np.ascontiguousarray(W[b.offsets[i]:b.offsets[i + 1]])
        tg = np.sort(np.random.default_rng(40 + i).choice(N, min(N, 1500), replace=False))
        Uo = _oracle_u_at(st, X, Wi, p, tg)
        _compare_structures(st, gs[i], tg)
        assert np.array_equal(gs[i]["hsrc"], st["hsrc"])
        Ui = Ub[b.offsets[i]:b.offsets[i + 1]].astype(np.float64)
        for r in range(2):
            e = rel(Ui[tg, r], Uo[:, r])
            print(f"[shape batched] instance {i} column {r}: {e:.2e}", flush=True)
            assert e < 1e-5
