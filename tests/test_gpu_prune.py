"""Pruning diagnostic (Table t:prune) on the GPU against the FP64 oracle
(needs an MI355X): for every point as a target, the nodes visited by Alg. 4
under neighbour pruning and under distance pruning, bit for bit, on the
paper's three point sets (curve, Gaussian, hypersphere) in several
dimensions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth
from tests.test_gpu_parity import gparams

pytestmark = pytest.mark.gpu

GEN = {"curve": synth.curve_points, "gaussian": synth.gaussian_points, "sphere": synth.sphere_points}


@pytest.mark.parametrize("kind,d", [("curve", 2), ("gaussian", 4), ("sphere", 4), ("curve", 32),
                                    ("sphere", 32), ("gaussian", 256)])
def test_prune_visits_bit_exact(kind, d):
    import torch
    from paper_1410_0260_amd import askit as A
    N, m, kappa = 4096, 64, 32
    X = GEN[kind](N, d, 11 + d)
    p = O.Params(m=m, kappa=kappa, smax=16, ell=36, tau=1e-3, h=1.0, seed=1)
    h = A.setup(torch.from_numpy(X).cuda(), gparams(p))
    vk, vd = h.pruning_visits()
    vk, vd = vk.cpu().numpy(), vd.cpu().numpy()
    g = h.structures()
    h.close()
    idx, _ = O.knn(X, X, kappa, exclude_self=True)
    nodes, perm = O.tree(X, m)
    assert np.array_equal(g["perm"], perm) and np.array_equal(g["knn_idx"], idx)
    iperm = np.empty(N, np.int32)
    iperm[perm] = np.arange(N, dtype=np.int32)
    ok, od, _, _ = O.prune_visits(X, perm, nodes, np.concatenate([iperm[:, None], iperm[idx]], axis=1))
    print(f"\n[prune] {kind} {d}-D: visited {100 * vk.mean() / len(nodes):.1f}% (kappa) "
          f"{100 * vd.mean() / len(nodes):.1f}% (distance)", flush=True)
    assert np.array_equal(vk, ok)
    assert np.array_equal(vd, od)
