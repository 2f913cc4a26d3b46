"""The paper's approximate neighbour search (iterated random projection trees,
Sec. 2.2) on the GPU against the FP64 oracle (needs an MI355X): ids and FP64
distances bit for bit, for several shapes, leaf sizes and round counts; and
ASKIT set up on those lists (askit_setup_with_knn) against the oracle run on
the same lists."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth
from tests.gpu_common import rel, slab_lists
from tests.test_gpu_parity import gparams

pytestmark = pytest.mark.gpu

CASES = [
    # N, d, q, comps, kappa, leaf, rounds, seed
    (3000, 8, 3, 3, 10, 64, 3, 7),
    (4999, 24, 4, 5, 16, 100, 5, 11),      # ragged leaves (N not a power of two)
    (2048, 64, 8, 4, 32, 130, 2, 13),
    (1500, 100, 5, 2, 8, 40, 4, 17),        # d above 64: several direction words
    (700, 3, 2, 2, 5, 700, 1, 19),           # one leaf: the exact lists
]


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}-d{c[1]}-k{c[4]}-leaf{c[5]}-r{c[6]}" for c in CASES])
def test_rpknn_bit_exact(case):
    import torch
    from paper_1410_0260_amd import askit as A
    N, d, q, comps, kappa, leaf, rounds, seed = case
    X = synth.mixture_points(N, d, q, comps, 1e-3, 50 + N)
    oi, od = O.rpknn(X, kappa, leaf, rounds, seed)
    gi, gd = A.knn_rptree(torch.from_numpy(X).cuda(), kappa, leaf, rounds, seed)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    ei, _ = O.knn(X, X, kappa, exclude_self=True)
    hit = np.mean([len(set(oi[i]) & set(ei[i])) for i in range(N)]) / kappa
    print(f"\n[rpknn] N={N} d={d} kappa={kappa} leaf={leaf} rounds={rounds}: hit rate {hit:.3f}", flush=True)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd, od)


def test_askit_on_approximate_lists():
    import torch
    from paper_1410_0260_amd import askit as A
    N, d = 6000, 12
    X = synth.mixture_points(N, d, 4, 4, 1e-3, 123)
    W = synth.weights(N, 2, 124)
    p = O.Params(m=128, kappa=16, smax=48, ell=68, tau=1e-6, h=0.9, seed=5)
    ki, kd = O.rpknn(X, p.kappa, 64, 2, 31)
    st = O.run_askit(X, W, p, record=True, knn_lists=(ki, kd))
    Xd = torch.from_numpy(X).cuda()
    gi, _ = A.knn_rptree(Xd, p.kappa, 64, 2, 31)
    h = A.setup_with_knn(Xd, gi, gparams(p))
    h.update_weights(torch.from_numpy(W).cuda())
    U = h.evaluate().cpu().numpy().astype(np.float64)
    g = h.structures()
    h.close()
    assert np.array_equal(g["knn_idx"], ki) and np.array_equal(g["knn_d"], kd)
    assert np.array_equal(g["perm"], st["perm"])
    for a in range(1, len(st["nodes"])):
        k = st["sk"].k[a]
        assert g["k"][a] == k and np.array_equal(g["S"][a, :k], st["sk"].S[a, :k]), f"node {a}"
    near, far = slab_lists(g, N)
    for o in range(0, N, 7):
        pos = st["iperm"][o]
        assert near[pos] == sorted(st["ev"].near[o].tolist()) and far[pos] == sorted(st["ev"].far[o].tolist())
    for r in range(2):
        assert rel(U[:, r], st["ev"].U[:, r]) < 1e-5


def test_rpknn_rejects_small_leaves():
    import torch
    from paper_1410_0260_amd import askit as A
    X = torch.from_numpy(synth.mixture_points(1000, 4, 2, 2, 1e-3, 9)).cuda()
    with pytest.raises(A.AskitError) as ei:
        A.knn_rptree(X, 16, 20, 1, 0)          # leaves of 15-20 points cannot hold 16 neighbours
    assert ei.value.code == A.ERR_INVALID_ARG
