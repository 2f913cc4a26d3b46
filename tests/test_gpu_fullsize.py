"""Parity at the full size of the 2^20-point, 64-dimensional workload, in the
launch configuration the benchmark times (same parameters, one RHS), on
outputs the FP64 oracle can compute one by one:

  * the whole tree (permutation and every node) -- the oracle builds it in full;
  * the kNN lists of sampled points (oracle exhaustive search per point), and
    of 256 new points;
  * for a sampled leaf beta: its node list (Alg. 2, leaf rule), sampled rows
    (Eq. e:sk_targets), skeleton and P (Alg. 3), and its skeleton weights;
  * the interaction lists of sampled targets (Alg. 4 / Eq. e:prune);
  * u for weights carried by beta alone.  Every other node then has zero
    skeleton weights, so for a target whose near set holds beta the result is
    beta's direct sum, and for a target that prunes beta itself it is the sum
    over beta's skeleton with w~_beta -- both computed by the oracle from its
    own tree, neighbours and skeleton of beta.  Targets that prune a proper
    ancestor of beta need that ancestor's skeleton and are not compared.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth

pytestmark = pytest.mark.gpu

U_TOL = 1e-5


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def full():
    import torch
    from paper_1410_0260_amd import askit as A
    wl = synth.fp32_1m()
    p = O.Params.from_workload(wl)
    _log(f"\n[fullsize] {wl.name}: oracle tree")
    X = synth.points(wl)
    N = wl.N
    nodes, perm = O.tree(X, p.m)
    iperm = np.empty(N, np.int32)
    iperm[perm] = np.arange(N, dtype=np.int32)
    rng = np.random.default_rng(2024)
    # beta: the leaf holding a random point; sigma: its sibling (a leaf too)
    pos0 = int(iperm[rng.integers(N)])
    beta = next(a for a in range(len(nodes)) if nodes[a]["left"] < 0
                and nodes[a]["lo"] <= pos0 < nodes[a]["hi"])
    par = nodes[beta]["parent"]
    sigma = nodes[par]["left"] if nodes[par]["right"] == beta else nodes[par]["right"]
    assert nodes[sigma]["left"] < 0
    bpts = perm[nodes[beta]["lo"]:nodes[beta]["hi"]]
    spts = rng.choice(perm[nodes[sigma]["lo"]:nodes[sigma]["hi"]], 192, replace=False)
    rpts = rng.choice(N, 64, replace=False)
    Wb = np.zeros((N, 1), np.float32)
    Wb[bpts, 0] = synth.weights(len(bpts), 1, 31)[:, 0]
    Yq = synth.queries(wl, 256, 77)

    _log("[fullsize] HIP setup + update + evaluate")
    h = A.setup(torch.from_numpy(X).cuda(), A.params_from_workload(wl))
    h.update_weights(torch.from_numpy(Wb).cuda())
    U = h.evaluate().cpu().numpy().astype(np.float64)[:, 0]
    torch.cuda.synchronize()
    g = h.structures()
    qi, qd = h.query_neighbors(torch.from_numpy(Yq).cuda())
    g["qidx"], g["qd"] = qi.cpu().numpy(), qd.cpu().numpy()
    h.close()
    # rows whose filter output overflowed (the re-filtered path): up to 64 of them
    retry_pos = g["knn_retry"]
    pick = rng.choice(len(retry_pos), min(64, len(retry_pos)), replace=False) if len(retry_pos) else []
    retry_ids = g["perm"][retry_pos[pick]].astype(np.int64) if len(retry_pos) else np.zeros(0, np.int64)
    rows = np.unique(np.concatenate([bpts, spts, rpts, retry_ids])).astype(np.int64)
    _log(f"[fullsize] oracle kNN of {len(rows)} points ({len(retry_ids)} of {len(retry_pos)} retried rows)")
    i1, d1 = O.knn(X[rows], X, p.kappa + 1, exclude_self=False)
    kidx = np.empty((len(rows), p.kappa), np.int32)
    kd = np.empty((len(rows), p.kappa))
    for r, o in enumerate(rows):
        keep = i1[r] != o
        kidx[r], kd[r] = i1[r][keep][:p.kappa], d1[r][keep][:p.kappa]
    _log(f"[fullsize] oracle kNN of {len(Yq)} new points")
    qidx_o, qd_o = O.knn(Yq, X, p.kappa, exclude_self=False)
    return dict(wl=wl, p=p, X=X, N=N, nodes=nodes, perm=perm, iperm=iperm, beta=beta, sigma=sigma,
                rows=rows, kidx=kidx, kd=kd, Wb=Wb, U=U, g=g, qidx=qidx_o, qd=qd_o, retry_ids=retry_ids)


def test_tree_full(full):
    g, nodes = full["g"], full["nodes"]
    assert np.array_equal(g["perm"], full["perm"])
    for f in ("lo", "hi", "level", "parent", "left", "right", "path"):
        assert np.array_equal(g["nodes"][f], nodes[f])


def test_knn_sampled(full):
    g, rows = full["g"], full["rows"]
    assert np.array_equal(g["knn_idx"][rows], full["kidx"])
    assert np.array_equal(g["knn_d"][rows], full["kd"])


def test_knn_retried_rows_covered(full):
    """At this size some rows' window bound lets more than the filter's
    capacity through; the sampled rows above include up to 64 of them."""
    assert full["g"]["info"]["knn_retry_rows"] == len(full["g"]["knn_retry"]) > 0
    assert np.isin(full["retry_ids"], full["rows"]).all() and len(full["retry_ids"]) > 0


def test_query_knn(full):
    """256 new points, through the sampled-threshold search at full size."""
    assert np.array_equal(full["g"]["qidx"], full["qidx"])
    assert np.array_equal(full["g"]["qd"], full["qd"])


@pytest.fixture(scope="module")
def beta_chain(full):
    """Oracle node list, sampled rows, skeleton and skeleton weights of beta
    alone: a two-node tree (the root, then beta) carries beta's level and
    path, so the oracle routines treat it exactly as in the whole tree."""
    p, N, beta = full["p"], full["N"], full["beta"]
    nd = full["nodes"][beta]
    two = np.zeros(2, dtype=O.NODE_DTYPE)
    two[0] = (0, N, 0, -1, 1, 1, 0)
    two[1] = (nd["lo"], nd["hi"], nd["level"], 0, -1, -1, nd["path"])
    kidx = np.zeros((N, p.kappa), np.int32)
    kd = np.zeros((N, p.kappa))
    sel = np.searchsorted(full["rows"], full["perm"][nd["lo"]:nd["hi"]])
    kidx[full["rows"][sel]] = full["kidx"][sel]
    kd[full["rows"][sel]] = full["kd"][sel]
    nl_pos, nl_key, nl_cnt = O.node_lists(two, N, full["perm"], kidx, kd, p.ell)
    T, T_cnt = O.sample_rows(two, N, nl_pos, nl_cnt, p.ell, p.seed)
    sk = O.skeletonize(full["X"], full["perm"], two, T, T_cnt, None, p.h, p.smax, p.tau, p.m)
    Wtree = full["Wb"][full["perm"]].astype(np.float64)
    Wsk = O.upward(two, Wtree, sk, p.smax)
    return dict(nl_pos=nl_pos[1], nl_key=nl_key[1], nl_cnt=int(nl_cnt[1]), T=T[1], T_cnt=int(T_cnt[1]),
                k=int(sk.k[1]), S=sk.S[1], ncols=int(sk.ncols[1]), P=sk.proj(1),
                margin=min(sk.piv_margin[1], sk.rank_margin[1]), Wsk=Wsk[1, :, 0])


def test_beta_node_list_and_rows(full, beta_chain):
    g, b, o = full["g"], full["beta"], beta_chain
    c = o["nl_cnt"]
    assert g["nl_cnt"][b] == c
    assert np.array_equal(g["nl_pos"][b, :c], o["nl_pos"][:c])
    assert np.array_equal(g["nl_key"][b, :c], o["nl_key"][:c])
    t = o["T_cnt"]
    assert g["T_cnt"][b] == t
    assert np.array_equal(g["T"][b, :t], o["T"][:t])


def _pslot_offset(nodes, a, p, N):
    """Start of node a's P slot: slots are packed in node order, each
    k_cap x n_cap with n_cap the column count bound and k_cap the rank bound."""
    off = 0
    for c in range(1, a):
        n_c = nodes[c]["hi"] - nodes[c]["lo"]
        ncap = n_c if nodes[c]["left"] < 0 else 2 * p.smax
        kcap = min(p.smax, min(p.ell, N - n_c), ncap)
        off += kcap * ncap
    return off


def test_beta_skeleton_and_projection(full, beta_chain):
    g, b, o, p = full["g"], full["beta"], beta_chain, full["p"]
    k = o["k"]
    same = g["k"][b] == k and np.array_equal(g["S"][b, :k], o["S"][:k])
    assert same or o["margin"] < 1e-10
    assert same, "certified near-tie at beta (none expected)"
    assert g["ncols"][b] == o["ncols"]
    n = o["ncols"]
    off = _pslot_offset(full["nodes"], b, p, full["N"])
    Pg = g["P"][off:off + k * (n - k)].reshape(k, n - k)
    assert np.linalg.norm(Pg - o["P"]) <= 1e-5 * max(1.0, np.linalg.norm(o["P"]))
    ref = o["Wsk"][:k]
    assert np.linalg.norm(g["Wsk"][b, :k, 0] - ref) <= 1e-5 * max(1.0, np.linalg.norm(ref))


def _gpu_lists(g, pos):
    """Near and far node ids of the target at tree position pos, read from
    the slab holding it (slabs are 64 consecutive positions of one leaf)."""
    ptr, node, mask, row0 = g["slab_ptr"], g["slab_node"], g["slab_mask"], g["slab_row0"]
    ns = len(row0)
    order = np.argsort(row0, kind="stable")
    s = int(order[np.searchsorted(row0[order], pos, side="right") - 1])
    bit = np.uint64(1) << np.uint64(pos - row0[s])
    out = []
    for lo, hi in ((ptr[s], ptr[s + 1]), (ptr[ns + 1 + s], ptr[ns + 2 + s])):
        out.append(sorted(int(node[e]) for e in range(lo, hi) if mask[e] & bit))
    return out


@pytest.fixture(scope="module")
def targets(full, beta_chain):
    """Oracle Alg. 4 on the sampled targets with weights on beta only and
    beta's oracle skeleton (all other skeletons are empty: their weights are 0)."""
    p, N, nodes = full["p"], full["N"], full["nodes"]
    nn = len(nodes)
    tg = full["rows"]
    nb = np.empty((len(tg), p.kappa + 1), np.int32)
    nb[:, 0] = full["iperm"][tg]
    nb[:, 1:] = full["iperm"][full["kidx"]]
    b, o = full["beta"], beta_chain
    S = np.full((nn, p.smax), -1, np.int32)
    k = np.zeros(nn, np.int32)
    S[b], k[b] = o["S"], o["k"]
    sk = O.Skeletons(k, S, None, None, None, None, None, 0)
    Wsk = np.zeros((nn, p.smax, 1))
    Wsk[b, :, 0] = o["Wsk"]
    ev = O.evaluate(full["X"][tg], nb, full["X"], full["perm"], nodes, None, p.h, full["Wb"], sk, Wsk,
                    p.smax, record=True)
    return tg, ev


def test_interaction_lists_sampled(full, targets):
    tg, ev = targets
    g = full["g"]
    for r, o in enumerate(tg):
        near, far = _gpu_lists(g, int(full["iperm"][o]))
        assert near == sorted(ev.near[r].tolist()), f"target {o}"
        assert far == sorted(ev.far[r].tolist()), f"target {o}"


def test_u_beta_weights(full, targets):
    tg, ev = targets
    b = full["beta"]
    is_near = np.array([b in ev.near[r] for r in range(len(tg))])
    is_far = np.array([b in ev.far[r] for r in range(len(tg))])
    Ug = full["U"][tg]
    Uo = ev.U[:, 0]
    _log(f"[fullsize] targets: {is_near.sum()} with beta near, {is_far.sum()} with beta pruned")
    assert is_near.sum() >= 256 and is_far.sum() >= 8
    for sel in (is_near, is_far):
        assert np.linalg.norm(Ug[sel] - Uo[sel]) <= U_TOL * np.linalg.norm(Uo[sel])


# ---------------------------------------------------------------------------
# Against the full FP64 oracle run of this workload (tests/golden/, written by
# tests/golden/make_fullsize_golden.py, which calls only the oracle): u and its
# near-field part at 10,000 seeded targets, their interaction lists, ~200
# nodes' skeletons on every level, and P, column order and skeleton weights of
# 8 nodes.
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "fullsize_fp32_1m_h1.npz")


@pytest.fixture(scope="module")
def gold():
    import torch
    from paper_1410_0260_amd import askit as A
    z = dict(np.load(GOLDEN))
    wl = synth.fp32_1m()
    assert float(z["h"]) == wl.h
    X = synth.points(wl)
    W = synth.weights(wl.N, wl.R, wl.seed)
    _log("\n[fullsize-oracle] HIP setup + update + evaluate with the workload's weights")
    h = A.setup(torch.from_numpy(X).cuda(), A.params_from_workload(wl))
    h.update_weights(torch.from_numpy(W).cuda())
    U, Un = h.evaluate_parts()
    torch.cuda.synchronize()
    g = h.structures()
    h.close()
    g["U"] = U.cpu().numpy().astype(np.float64)[:, 0]
    g["Un"] = Un.cpu().numpy().astype(np.float64)[:, 0]
    return wl, z, g


def test_fullsize_oracle_u(gold):
    wl, z, g = gold
    tg = z["targets"]
    e = float(np.linalg.norm(g["U"][tg] - z["u"]) / np.linalg.norm(z["u"]))
    en = float(np.linalg.norm(g["Un"][tg] - z["u_near"]) / np.linalg.norm(z["u_near"]))
    eps_gpu = float(np.linalg.norm(g["U"][tg] - z["u_direct"]) / np.linalg.norm(z["u_direct"]))
    _log(f"[fullsize-oracle] u vs oracle {e:.2e}, near part {en:.2e}; eps vs FP64 direct: GPU {eps_gpu:.4f}, "
         f"oracle {float(z['eps']):.4f}")
    assert e < U_TOL and en < U_TOL
    assert abs(eps_gpu - float(z["eps"])) <= 1e-4 * float(z["eps"]) + 1e-6


def test_fullsize_oracle_lists(gold):
    wl, z, g = gold
    N = wl.N
    iperm = np.empty(N, np.int64)
    iperm[g["perm"]] = np.arange(N)
    for r, o in enumerate(z["targets"]):
        near, far = _gpu_lists(g, int(iperm[o]))
        for ids, c, s1, s2 in ((near, "near_cnt", "near_s1", "near_s2"), (far, "far_cnt", "far_s1", "far_s2")):
            a = np.array(ids, np.int64)
            assert (len(a), int(a.sum()), int((a * a).sum())) == (int(z[c][r]), int(z[s1][r]), int(z[s2][r])), \
                f"target {o}"


def test_fullsize_oracle_nodes(gold):
    wl, z, g = gold
    ties = 0
    for r, a in enumerate(z["nodes"]):
        k = int(z["k"][r])
        same = g["k"][a] == k and np.array_equal(g["S"][a, :k], z["S"][r, :k])
        if not same:
            assert min(z["piv_margin"][r], z["rank_margin"][r]) < 1e-10, f"node {a}"
            ties += 1
    assert ties == 0


def test_fullsize_oracle_projections(gold):
    wl, z, g = gold
    p = O.Params.from_workload(wl)
    V = np.random.default_rng(20141003).standard_normal((int(g["info"]["ncol_max"]), z["p_sketch"].shape[2]))
    for r, a in enumerate(z["p_nodes"]):
        k, n = int(g["k"][a]), int(z["p_ncols"][r])
        assert g["ncols"][a] == n and np.array_equal(g["colperm"][a, :n], z["p_colperm"][r, :n]), f"node {a}"
        off = _pslot_offset(g["nodes"], a, p, wl.N)
        Pg = g["P"][off:off + k * (n - k)].reshape(k, n - k).astype(np.float64)
        sk = Pg @ V[:n - k]
        ref = z["p_sketch"][r, :k]
        assert np.linalg.norm(sk - ref) <= 1e-5 * max(1.0, np.linalg.norm(ref)), f"node {a}"
        assert abs(np.linalg.norm(Pg) - z["p_fro"][r]) <= 1e-5 * max(1.0, z["p_fro"][r]), f"node {a}"
        w = z["wsk"][r, :k]
        assert np.linalg.norm(g["Wsk"][a, :k, 0] - w) <= 1e-5 * max(1.0, np.linalg.norm(w)), f"node {a}"
