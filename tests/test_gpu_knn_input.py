"""Given neighbour lists (askit_setup_with_knn) and the near-field part of u
(askit_evaluate_parts), against the FP64 oracle (needs an MI355X).

The paper's driver takes N(X) as an input (Alg. 5): with the same lists the
oracle and the library must build the same tree, node lists, sampled rows,
skeletons and interaction lists, bit for bit, and the same u within 1e-5.
The lists here are deliberately not the exact ones: each row keeps a seeded
subset of kappa of the kappa + 8 nearest points, handed over in a shuffled
order, so that the library's own search could not produce them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth
from tests.gpu_common import rel, slab_lists
from tests.test_gpu_parity import CASES, U_TOL, gparams

pytestmark = pytest.mark.gpu


def inexact_lists(X, kappa, seed):
    """Rows of kappa ids drawn from each point's kappa + 8 nearest (oracle
    search), in a shuffled order; also sorted by (distance, id) for the oracle."""
    N = len(X)
    extra = min(8, N - 1 - kappa)
    i1, d1 = O.knn(X, X, kappa + extra, exclude_self=True)
    rng = np.random.default_rng(seed)
    given = np.empty((N, kappa), np.int32)
    srt_i = np.empty((N, kappa), np.int32)
    srt_d = np.empty((N, kappa))
    for r in range(N):
        pick = np.sort(rng.choice(kappa + extra, kappa, replace=False))
        ids, ds = i1[r, pick], d1[r, pick]
        order = np.lexsort((ids, ds))
        srt_i[r], srt_d[r] = ids[order], ds[order]
        given[r] = rng.permutation(ids)
    return given, srt_i, srt_d


@pytest.fixture(scope="module", params=["small-fp64", "varh", "filter-path"])
def given(request):
    import torch
    from paper_1410_0260_amd import askit as A
    N, d, q, comps, p = CASES[request.param]
    X = synth.mixture_points(N, d, q, comps, 1e-3, 300 + N)
    W = synth.weights(N, 2, 300 + N)
    print(f"\n[knn-input {request.param}] N={N} d={d}", flush=True)
    knn_given, kidx, kd = inexact_lists(X, p.kappa, N)
    st = O.run_askit(X, W, p, record=True, knn_lists=(kidx, kd))
    h = A.setup_with_knn(torch.from_numpy(X).cuda(), torch.from_numpy(knn_given).cuda(), gparams(p))
    h.update_weights(torch.from_numpy(W).cuda())
    U, Un = h.evaluate_parts()
    U2 = h.evaluate()
    torch.cuda.synchronize()
    g = h.structures()
    g["U"], g["Unear"], g["U2"] = (U.cpu().numpy().astype(np.float64), Un.cpu().numpy().astype(np.float64),
                                   U2.cpu().numpy().astype(np.float64))
    h.close()
    return request.param, X, W, p, st, g


def test_given_lists_kept(given):
    name, X, W, p, st, g = given
    assert np.array_equal(g["knn_idx"], st["knn_idx"])
    assert np.array_equal(g["knn_d"], st["knn_d"])
    if p.bw_neighbor:
        assert np.array_equal(g["hsrc"], st["hsrc"])


def test_downstream_structures_bit_exact(given):
    name, X, W, p, st, g = given
    assert np.array_equal(g["perm"], st["perm"])
    assert np.array_equal(g["nl_cnt"], st["nl_cnt"])
    assert np.array_equal(g["T_cnt"], st["T_cnt"])
    for a in range(1, len(st["nodes"])):
        c, t = st["nl_cnt"][a], st["T_cnt"][a]
        assert np.array_equal(g["nl_pos"][a, :c], st["nl_pos"][a, :c]), f"node {a}"
        assert np.array_equal(g["nl_key"][a, :c], st["nl_key"][a, :c]), f"node {a}"
        assert np.array_equal(g["T"][a, :t], st["T"][a, :t]), f"node {a}"
        k = st["sk"].k[a]
        assert g["k"][a] == k and np.array_equal(g["S"][a, :k], st["sk"].S[a, :k]), f"node {a}"
    near, far = slab_lists(g, len(X))
    for o in range(len(X)):
        pos = st["iperm"][o]
        assert near[pos] == sorted(st["ev"].near[o].tolist()), f"target {o}"
        assert far[pos] == sorted(st["ev"].far[o].tolist()), f"target {o}"


def test_u_and_near_part_match_oracle(given):
    name, X, W, p, st, g = given
    assert np.array_equal(g["U"], g["U2"])        # the near part is a prefix of the same sums
    for r in range(W.shape[1]):
        e = rel(g["U"][:, r], st["ev"].U[:, r])
        en = rel(g["Unear"][:, r], st["ev"].Unear[:, r])
        print(f"[knn-input {name}] column {r}: u {e:.2e}, near part {en:.2e}", flush=True)
        assert e < U_TOL and en < U_TOL


def test_given_lists_rejected():
    import torch
    from paper_1410_0260_amd import askit as A
    N, d = 600, 6
    X = synth.mixture_points(N, d, 3, 2, 1e-3, 61)
    p = O.Params(m=64, kappa=6, smax=16, ell=36, tau=1e-6, h=0.8, seed=1)
    good, _, _ = inexact_lists(X, p.kappa, 5)
    Xd = torch.from_numpy(X).cuda()
    for bad_case in ("self", "range", "repeat"):
        bad = good.copy()
        if bad_case == "self":
            bad[17, 2] = 17
        elif bad_case == "range":
            bad[3, 0] = N
        else:
            bad[9, 4] = bad[9, 1]
        with pytest.raises(A.AskitError) as ei:
            A.setup_with_knn(Xd, torch.from_numpy(bad).cuda(), gparams(p))
        assert ei.value.code == A.ERR_INVALID_ARG
