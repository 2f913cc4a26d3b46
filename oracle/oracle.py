"""Python front end of the FP64 ASKIT oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  It loads `liboracle.so`, built from
`askit_oracle.c` by `build.py` with gcc, and shares nothing with the HIP
library.

`run_askit` strings the oracle's stages together in the order of the
ASKIT driver (Alg. 5): neighbours, tree, node lists (Alg. 2), sampled
rows (Eq. e:sk_targets), skeletonization (Alg. 3), skeleton weights and
evaluation (Alg. 4).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

NODE_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("level", "<i4"), ("parent", "<i4"),
                       ("left", "<i4"), ("right", "<i4"), ("path", "<i8")])


def lib():
    global _lib
    if _lib is None:
        # ASKIT_ORACLE_ASAN=1: the sanitizer build (the process must preload
        # the ASan runtime)
        asan = os.environ.get("ASKIT_ORACLE_ASAN") == "1"
        path = _build.build_asan(force=False) if asan else _build.build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32, f64, u64 = C.c_int64, C.c_int, C.c_double, C.c_uint64
        L.or_sizeof_node.restype = i32
        L.or_direct.argtypes = [P, i64, P, i64, i32, P, i32, P, f64, P]
        L.or_knn.argtypes = [P, i64, P, i64, i32, i32, i32, P, P]
        L.or_bandwidth.argtypes = [P, i64, i32, i32, P]
        L.or_rpknn.argtypes = [P, i64, i32, i32, i32, i32, u64, P, P]
        L.or_prune_visits.argtypes = [P, i64, i32, P, P, i64, P, i32, P, P, P, P]
        L.or_tree_count.argtypes = [i64, i32]
        L.or_tree_count.restype = i64
        L.or_tree.argtypes = [P, i64, i32, i32, P, i64, P]
        L.or_node_lists.argtypes = [P, i64, i64, P, P, P, i32, i32, P, P, P]
        L.or_splitmix64.argtypes = [u64, u64]
        L.or_splitmix64.restype = u64
        L.or_sample_rows.argtypes = [P, i64, i64, P, P, i32, u64, P, P]
        L.or_gauss_matrix.argtypes = [P, i32, P, i32, P, i32, P, f64, P]
        L.or_id.argtypes = [P, i32, i32, i32, f64, P, P, P, P, P, P]
        L.or_skeletonize.argtypes = [P, i64, i32, P, P, i64, P, P, i32, P, f64, i32, f64, i32,
                                     P, P, P, P, P, P, P]
        L.or_upward.argtypes = [P, i64, P, i32, i32, P, P, i32, P, P, P]
        L.or_evaluate.argtypes = [P, i64, P, i32, P, i32, P, P, P, f64, P, i32, P, P, i32, P,
                                  P, P, P, P, i32, P, P, i32, i32]
        for f in ("or_direct", "or_knn", "or_rpknn", "or_prune_visits", "or_bandwidth", "or_tree", "or_node_lists",
                  "or_sample_rows", "or_gauss_matrix", "or_id", "or_skeletonize", "or_upward",
                  "or_evaluate"):
            getattr(L, f).restype = i32
        assert L.or_sizeof_node() == NODE_DTYPE.itemsize
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ---------------------------------------------------------------- stages
def direct(T, X, W, h, hsrc=None):
    """u(t) = sum_j exp(-|t - x_j|^2 / (2 h_j^2)) w_j in FP64 (Eq. e:problem)."""
    T, X = _f32(T), _f32(X)
    W = _f32(W if W.ndim == 2 else W[:, None])
    hs = None if hsrc is None else np.ascontiguousarray(hsrc, dtype=np.float64)
    U = np.empty((T.shape[0], W.shape[1]), dtype=np.float64)
    _check(lib().or_direct(_p(T), T.shape[0], _p(X), X.shape[0], X.shape[1], _p(W), W.shape[1],
                           _p(hs), float(h), _p(U)), "direct")
    return U


def knn(Q, X, kappa, exclude_self):
    Q, X = _f32(Q), _f32(X)
    idx = np.empty((Q.shape[0], kappa), dtype=np.int32)
    dist = np.empty((Q.shape[0], kappa), dtype=np.float64)
    _check(lib().or_knn(_p(Q), Q.shape[0], _p(X), X.shape[0], X.shape[1], kappa,
                        1 if exclude_self else 0, _p(idx), _p(dist)), "knn")
    return idx, dist


def rpknn(X, kappa, leaf, rounds, seed):
    """Approximate kappa nearest neighbours by iterated random projection trees."""
    X = _f32(X)
    N = X.shape[0]
    idx = np.empty((N, kappa), dtype=np.int32)
    dist = np.empty((N, kappa), dtype=np.float64)
    _check(lib().or_rpknn(_p(X), N, X.shape[1], kappa, leaf, rounds, C.c_uint64(seed & (2**64 - 1)),
                          _p(idx), _p(dist)), "rpknn")
    return idx, dist


def bandwidth(dist, b):
    dist = np.ascontiguousarray(dist, dtype=np.float64)
    h = np.empty(dist.shape[0], dtype=np.float64)
    _check(lib().or_bandwidth(_p(dist), dist.shape[0], dist.shape[1], b, _p(h)), "bandwidth")
    return h


def tree_count(N, m):
    return int(lib().or_tree_count(N, m))


def tree(X, m):
    X = _f32(X)
    N = X.shape[0]
    nn = tree_count(N, m)
    nodes = np.zeros(nn, dtype=NODE_DTYPE)
    perm = np.empty(N, dtype=np.int32)
    _check(lib().or_tree(_p(X), N, X.shape[1], m, _p(nodes), nn, _p(perm)), "tree")
    return nodes, perm


def node_lists(nodes, N, perm, knn_idx, knn_d, ell):
    nn = len(nodes)
    kappa = knn_idx.shape[1]
    nl_pos = np.full((nn, ell), -1, dtype=np.int32)
    nl_key = np.zeros((nn, ell), dtype=np.float64)
    nl_cnt = np.zeros(nn, dtype=np.int32)
    _check(lib().or_node_lists(_p(nodes), nn, N, _p(np.ascontiguousarray(perm, np.int32)),
                               _p(np.ascontiguousarray(knn_idx, np.int32)),
                               _p(np.ascontiguousarray(knn_d, np.float64)), kappa, ell,
                               _p(nl_pos), _p(nl_key), _p(nl_cnt)), "node_lists")
    return nl_pos, nl_key, nl_cnt


def splitmix64(base, t):
    return int(lib().or_splitmix64(C.c_uint64(base & (2**64 - 1)), C.c_uint64(t)))


def sample_rows(nodes, N, nl_pos, nl_cnt, ell, seed):
    nn = len(nodes)
    T = np.full((nn, ell), -1, dtype=np.int32)
    T_cnt = np.zeros(nn, dtype=np.int32)
    _check(lib().or_sample_rows(_p(nodes), nn, N, _p(np.ascontiguousarray(nl_pos, np.int32)),
                                _p(np.ascontiguousarray(nl_cnt, np.int32)), ell,
                                C.c_uint64(seed & (2**64 - 1)), _p(T), _p(T_cnt)), "sample_rows")
    return T, T_cnt


def gauss_matrix(X, rows, cols, h, hsrc=None):
    X = _f32(X)
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    G = np.empty((len(rows), len(cols)), dtype=np.float64)
    hs = None if hsrc is None else np.ascontiguousarray(hsrc, dtype=np.float64)
    _check(lib().or_gauss_matrix(_p(X), X.shape[1], _p(rows), len(rows), _p(cols), len(cols),
                                 _p(hs), float(h), _p(G)), "gauss_matrix")
    return G


@dataclass
class IDResult:
    k: int
    piv: np.ndarray        # all column pivots, skeleton = piv[:k]
    P: np.ndarray          # k x (cols - k)
    rdiag: np.ndarray      # R_tt, t < k
    piv_margin: float
    rank_margin: float


def interp_decomp(G, smax, tau):
    G = np.ascontiguousarray(G, dtype=np.float64)
    rows, cols = G.shape
    piv = np.empty(max(cols, 1), dtype=np.int32)
    kk = np.zeros(1, dtype=np.int32)
    P = np.zeros(max(1, min(smax, rows, cols) * cols), dtype=np.float64)
    rd = np.zeros(max(1, min(smax, rows, cols)), dtype=np.float64)
    pm = np.zeros(1)
    rm = np.zeros(1)
    _check(lib().or_id(_p(G), rows, cols, smax, float(tau), _p(piv), _p(kk), _p(P), _p(rd),
                       _p(pm), _p(rm)), "id")
    k = int(kk[0])
    return IDResult(k, piv[:cols].copy(), P[:k * (cols - k)].reshape(k, cols - k).copy(),
                    rd[:k].copy(), float(pm[0]), float(rm[0]))


@dataclass
class Skeletons:
    k: np.ndarray          # per node
    S: np.ndarray          # nn x smax tree positions
    colperm: np.ndarray    # nn x ncol_max
    ncols: np.ndarray
    P: np.ndarray          # nn x smax x ncol_max slots (row stride ncols-k)
    piv_margin: np.ndarray
    rank_margin: np.ndarray
    ncol_max: int

    def proj(self, a):
        k, n = int(self.k[a]), int(self.ncols[a])
        return self.P[a].reshape(-1)[:k * (n - k)].reshape(k, n - k)


def skeletonize(X, perm, nodes, T, T_cnt, hsrc, h, smax, tau, m):
    X = _f32(X)
    nn = len(nodes)
    ell = T.shape[1]
    ncol_max = max(m, 2 * smax)
    S = np.full((nn, smax), -1, dtype=np.int32)
    k = np.zeros(nn, dtype=np.int32)
    colperm = np.full((nn, ncol_max), -1, dtype=np.int32)
    ncols = np.zeros(nn, dtype=np.int32)
    P = np.zeros((nn, smax, ncol_max), dtype=np.float64)
    pm = np.full(nn, np.inf)
    rm = np.full(nn, np.inf)
    hs = None if hsrc is None else np.ascontiguousarray(hsrc, dtype=np.float64)
    _check(lib().or_skeletonize(_p(X), X.shape[0], X.shape[1], _p(np.ascontiguousarray(perm, np.int32)),
                                _p(nodes), nn, _p(np.ascontiguousarray(T, np.int32)),
                                _p(np.ascontiguousarray(T_cnt, np.int32)), ell, _p(hs), float(h),
                                smax, float(tau), ncol_max, _p(S), _p(k), _p(colperm), _p(ncols),
                                _p(P), _p(pm), _p(rm)), "skeletonize")
    return Skeletons(k, S, colperm, ncols, P, pm, rm, ncol_max)


def upward(nodes, Wtree, sk: Skeletons, smax):
    Wtree = np.ascontiguousarray(Wtree, dtype=np.float64)
    if Wtree.ndim == 1:
        Wtree = Wtree[:, None]
    R = Wtree.shape[1]
    nn = len(nodes)
    Wsk = np.zeros((nn, smax, R), dtype=np.float64)
    _check(lib().or_upward(_p(nodes), nn, _p(Wtree), R, smax, _p(sk.k), _p(sk.colperm),
                           sk.ncol_max, _p(sk.ncols), _p(sk.P), _p(Wsk)), "upward")
    return Wsk


@dataclass
class EvalResult:
    U: np.ndarray
    Unear: np.ndarray
    near: list            # per target: near leaf ids (visit order)
    far: list             # per target: pruned node ids (visit order)


def min_prune_level(nodes, prune_levels):
    """First level whose nodes may be pruned: 0 (every level) when
    prune_levels is 0, else the prune_levels deepest levels only."""
    if prune_levels <= 0:
        return 0
    return max(1, int(nodes["level"].max()) - prune_levels + 1)


def evaluate(Y, nb, X, perm, nodes, hsrc, h, W, sk: Skeletons, Wsk, smax, record=True, min_level=0):
    Y, X = _f32(Y), _f32(X)
    W = _f32(W if W.ndim == 2 else W[:, None])
    nb = np.ascontiguousarray(nb, dtype=np.int32)
    M, nnb = nb.shape
    R = W.shape[1]
    U = np.zeros((M, R))
    Un = np.zeros((M, R))
    depth = int(nodes["level"].max()) + 1
    near_cap = nnb + 1 if min_level == 0 else int((nodes["left"] < 0).sum())
    far_cap = (nnb + 1) * depth + 1 if min_level == 0 else len(nodes)
    nids = np.zeros((M, near_cap), np.int32) if record else None
    fids = np.zeros((M, far_cap), np.int32) if record else None
    ncnt = np.zeros(M, np.int32)
    fcnt = np.zeros(M, np.int32)
    hs = None if hsrc is None else np.ascontiguousarray(hsrc, dtype=np.float64)
    _check(lib().or_evaluate(_p(Y), M, _p(nb), nnb, _p(X), X.shape[1],
                             _p(np.ascontiguousarray(perm, np.int32)), _p(nodes), _p(hs), float(h),
                             _p(W), R, _p(sk.S), _p(sk.k), smax,
                             _p(np.ascontiguousarray(Wsk, np.float64)), _p(U), _p(Un),
                             _p(nids), _p(ncnt), near_cap if record else 0,
                             _p(fids), _p(fcnt), far_cap if record else 0, int(min_level)), "evaluate")
    near = [nids[i, :ncnt[i]].copy() for i in range(M)] if record else None
    far = [fids[i, :fcnt[i]].copy() for i in range(M)] if record else None
    return EvalResult(U, Un, near, far)


def prune_visits(X, perm, nodes, nb):
    """Per target (point i, original order; nb row i = position of i and of its
    neighbours): nodes visited by Alg. 4 under neighbour pruning and under
    distance pruning (Table t:prune), with the node centroids and squared radii."""
    X = _f32(X)
    N, d = X.shape
    nn = len(nodes)
    nb = np.ascontiguousarray(nb, dtype=np.int32)
    vk = np.zeros(N, np.int32)
    vd = np.zeros(N, np.int32)
    cen = np.zeros((nn, d))
    r2 = np.zeros(nn)
    _check(lib().or_prune_visits(_p(X), N, d, _p(np.ascontiguousarray(perm, np.int32)), _p(nodes), nn, _p(nb),
                                 nb.shape[1], _p(vk), _p(vd), _p(cen), _p(r2)), "prune_visits")
    return vk, vd, cen, r2


# ---------------------------------------------------------------- driver
@dataclass
class Params:
    m: int
    kappa: int
    smax: int
    ell: int
    tau: float
    h: float               # fixed bandwidth (ignored when bw_neighbor > 0)
    bw_neighbor: int = 0
    seed: int = 0
    prune_levels: int = 0  # > 0: only the prune_levels deepest levels may be pruned

    @staticmethod
    def from_workload(w):
        return Params(w.m, w.kappa, w.smax, w.ell_eff, w.tau, w.h, w.bw_neighbor, w.seed, w.prune_levels)


def setup(X, p: Params, knn_lists=None):
    """Tree, neighbours, node lists, sampled rows and skeletons (Alg. 5 lines 1-3)."""
    X = _f32(X)
    N = X.shape[0]
    if knn_lists is None:
        kidx, kd = knn(X, X, p.kappa, exclude_self=True)
    else:
        kidx, kd = knn_lists
    hsrc = bandwidth(kd, p.bw_neighbor) if p.bw_neighbor > 0 else None
    nodes, perm = tree(X, p.m)
    iperm = np.empty(N, np.int32)
    iperm[perm] = np.arange(N, dtype=np.int32)
    nl_pos, nl_key, nl_cnt = node_lists(nodes, N, perm, kidx, kd, p.ell)
    T, T_cnt = sample_rows(nodes, N, nl_pos, nl_cnt, p.ell, p.seed)
    sk = skeletonize(X, perm, nodes, T, T_cnt, hsrc, p.h, p.smax, p.tau, p.m)
    return dict(X=X, N=N, p=p, knn_idx=kidx, knn_d=kd, hsrc=hsrc, nodes=nodes, perm=perm,
                iperm=iperm, nl_pos=nl_pos, nl_key=nl_key, nl_cnt=nl_cnt, T=T, T_cnt=T_cnt,
                sk=sk)


def self_neighbours(st, targets_orig):
    """Neighbour positions {i} U N_i for targets given by original id."""
    t = np.asarray(targets_orig, dtype=np.int64)
    nb = np.empty((len(t), st["p"].kappa + 1), dtype=np.int32)
    nb[:, 0] = st["iperm"][t]
    nb[:, 1:] = st["iperm"][st["knn_idx"][t]]
    return nb


def run_askit(X, W, p: Params, targets=None, record=True, knn_lists=None):
    """Whole ASKIT (Alg. 5) in FP64; targets are original ids (default: all)."""
    st = setup(X, p, knn_lists)
    W = _f32(W if W.ndim == 2 else W[:, None])
    Wtree = W[st["perm"]].astype(np.float64)
    Wsk = upward(st["nodes"], Wtree, st["sk"], p.smax)
    tgt = np.arange(st["N"]) if targets is None else np.asarray(targets)
    nb = self_neighbours(st, tgt)
    ev = evaluate(st["X"][tgt], nb, st["X"], st["perm"], st["nodes"], st["hsrc"], p.h, W,
                  st["sk"], Wsk, p.smax, record=record, min_level=min_prune_level(st["nodes"], p.prune_levels))
    st.update(W=W, Wsk=Wsk, targets=tgt, ev=ev)
    return st


def query(st, Y, record=True):
    """Evaluation at new points (targets distinct from sources): neighbours of y
    among the sources, then Alg. 4 with Prune(alpha) <=> alpha holds none of them."""
    Y = _f32(Y)
    qi, qd = knn(Y, st["X"], st["p"].kappa, exclude_self=False)
    nb = st["iperm"][qi].astype(np.int32)
    ev = evaluate(Y, nb, st["X"], st["perm"], st["nodes"], st["hsrc"], st["p"].h, st["W"],
                  st["sk"], st["Wsk"], st["p"].smax, record=record,
                  min_level=min_prune_level(st["nodes"], st["p"].prune_levels))
    return qi, qd, ev
