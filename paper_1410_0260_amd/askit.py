"""Thin Python binding of the gfx950 ASKIT library (`libaskit.so`).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (CUDA/HIP tensors) and the
current stream; the library is called through its C ABI (include/askit.h).
Importing this module loads the library and fails loudly when it has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaskit.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_READY, ERR_UNSUPPORTED, ERR_BUSY = range(7)
PREC_FP32, PREC_BF16X3 = 0, 1
ABI_VERSION = 2

X_PERM, X_KNN_IDX, X_KNN_DIST, X_NODES, X_NLIST_POS, X_NLIST_KEY, X_NLIST_CNT = 1, 2, 3, 4, 5, 6, 7
X_ROWS, X_ROWS_CNT, X_SKEL, X_SKEL_K, X_COLPERM, X_NCOLS, X_PROJ, X_SKEL_W = 8, 9, 10, 11, 12, 13, 14, 15
X_SLAB_PTR, X_SLAB_NODE, X_SLAB_MASK, X_SLAB_ROW0, X_BANDWIDTH = 16, 17, 18, 19, 20
X_KNN_RETRY = 21

NODE_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("level", "<i4"), ("parent", "<i4"),
                       ("left", "<i4"), ("right", "<i4"), ("path", "<i8")])


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("abi_version", C.c_uint32),
                ("leaf_size", C.c_int32), ("kappa", C.c_int32), ("max_skeleton", C.c_int32),
                ("sample_rows", C.c_int32), ("id_tol", C.c_double), ("bandwidth", C.c_double),
                ("bw_neighbor", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("prune_levels", C.c_int32), ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int64), ("d", C.c_int32), ("kappa", C.c_int32), ("leaf_size", C.c_int32),
                ("max_skeleton", C.c_int32), ("sample_rows", C.c_int32), ("nrhs", C.c_int32),
                ("num_nodes", C.c_int32), ("num_leaves", C.c_int32), ("depth", C.c_int32),
                ("ncol_max", C.c_int32), ("num_slabs", C.c_int32), ("near_entries", C.c_int64),
                ("far_entries", C.c_int64), ("near_pairs", C.c_int64), ("far_pairs", C.c_int64),
                ("knn_uncertified_rows", C.c_int64), ("t_knn_ms", C.c_double),
                ("t_tree_ms", C.c_double), ("t_lists_ms", C.c_double), ("t_skel_ms", C.c_double),
                ("t_inter_ms", C.c_double), ("t_update_ms", C.c_double),
                ("t_knn_sweep_ms", C.c_double), ("t_qr_ms", C.c_double),
                ("t_knn_filter_ms", C.c_double), ("knn_filter_launches", C.c_int64),
                ("eval_pairs", C.c_int64), ("eval_chunks", C.c_int64), ("knn_retry_rows", C.c_int64),
                ("near_lists", C.c_int64), ("far_lists", C.c_int64), ("knn_tiles_swept", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class AskitError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"askit error {code}: {msg}")
        self.code = code


_lib = None

EXPORTED = ["askit_params_default", "askit_setup", "askit_setup_with_knn", "askit_update_weights",
            "askit_evaluate", "askit_evaluate_parts", "askit_evaluate_weights_noalloc", "askit_knn_rptree",
            "askit_pruning_visits", "askit_query", "askit_query_neighbors", "askit_destroy", "askit_last_error", "askit_get_info",
            "askit_export"]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.askit_params_default.argtypes = [C.POINTER(Params)]
        L.askit_setup.argtypes = [P, i64, i32, i64, C.POINTER(Params), P, C.POINTER(P)]
        L.askit_update_weights.argtypes = [P, P, i64, i32, P]
        L.askit_setup_with_knn.argtypes = [P, i64, i32, i64, P, i64, C.POINTER(Params), P, C.POINTER(P)]
        L.askit_evaluate.argtypes = [P, P, i64, P]
        L.askit_evaluate_parts.argtypes = [P, P, i64, P, i64, P]
        L.askit_evaluate_weights_noalloc.argtypes = [P, P, i64, i32, P, i64, P]
        L.askit_knn_rptree.argtypes = [P, i64, i32, i64, i32, i32, i32, C.c_uint64, P, P, P]
        L.askit_pruning_visits.argtypes = [P, P, P, P]
        L.askit_query.argtypes = [P, P, i64, i64, P, i64, P]
        L.askit_query_neighbors.argtypes = [P, P, i64, i64, P, P, P]
        L.askit_destroy.argtypes = [P]
        L.askit_destroy.restype = None
        L.askit_last_error.restype = C.c_char_p
        L.askit_get_info.argtypes = [P, C.POINTER(Info)]
        L.askit_export.argtypes = [P, i32, P, C.c_size_t, C.POINTER(C.c_size_t)]
        for f in EXPORTED:
            if f not in ("askit_destroy", "askit_last_error"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise AskitError(rc, lib().askit_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().askit_params_default(C.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def params_from_workload(w, precision=PREC_FP32) -> Params:
    return default_params(leaf_size=w.m, kappa=w.kappa, max_skeleton=w.smax, sample_rows=w.ell_eff,
                          id_tol=w.tau, bandwidth=w.h if w.h > 0 else 1.0,
                          bw_neighbor=w.bw_neighbor, precision=precision, seed=w.seed,
                          prune_levels=w.prune_levels)


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(torch, a):
    t = a if torch.is_tensor(a) else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    t = t.to(device="cuda", dtype=torch.float32)
    if t.dim() == 1:
        t = t[:, None]
    return t.contiguous()


@dataclass
class Handle:
    ptr: C.c_void_p
    N: int
    d: int
    nrhs: int = 0

    # -------------------------------------------------------------- calls
    def update_weights(self, W):
        import torch
        Wd = _dev_f32(torch, W)
        assert Wd.shape[0] == self.N
        _check(lib().askit_update_weights(self.ptr, C.c_void_p(Wd.data_ptr()), Wd.stride(0),
                                          Wd.shape[1], _stream(torch)))
        self.nrhs = Wd.shape[1]

    def evaluate(self, out=None):
        import torch
        U = out if out is not None else torch.empty((self.N, self.nrhs), device="cuda",
                                                     dtype=torch.float32)
        _check(lib().askit_evaluate(self.ptr, C.c_void_p(U.data_ptr()), U.stride(0), _stream(torch)))
        return U

    def evaluate_parts(self):
        """(u, near-field part of u) at every point."""
        import torch
        U = torch.empty((self.N, self.nrhs), device="cuda", dtype=torch.float32)
        Un = torch.empty((self.N, self.nrhs), device="cuda", dtype=torch.float32)
        _check(lib().askit_evaluate_parts(self.ptr, C.c_void_p(U.data_ptr()), U.stride(0),
                                          C.c_void_p(Un.data_ptr()), Un.stride(0), _stream(torch)))
        return U, Un

    def evaluate_weights_noalloc(self, W, out=None):
        """u = K w for W through the entry point that allocates nothing."""
        import torch
        Wd = _dev_f32(torch, W)
        assert Wd.shape[0] == self.N
        U = out if out is not None else torch.empty((self.N, Wd.shape[1]), device="cuda", dtype=torch.float32)
        _check(lib().askit_evaluate_weights_noalloc(self.ptr, C.c_void_p(Wd.data_ptr()), Wd.stride(0),
                                                    Wd.shape[1], C.c_void_p(U.data_ptr()), U.stride(0),
                                                    _stream(torch)))
        return U

    def query(self, Y, out=None):
        import torch
        Yd = _dev_f32(torch, Y)
        M = Yd.shape[0]
        U = out if out is not None else torch.empty((M, self.nrhs), device="cuda", dtype=torch.float32)
        _check(lib().askit_query(self.ptr, C.c_void_p(Yd.data_ptr()), M, Yd.stride(0),
                                 C.c_void_p(U.data_ptr()), U.stride(0), _stream(torch)))
        return U

    def query_neighbors(self, Y):
        """(ids, squared distances) of the kappa nearest sources of each row of Y."""
        import torch
        kappa = self.info()["kappa"]
        Yd = _dev_f32(torch, Y)
        M = Yd.shape[0]
        idx = torch.empty((M, kappa), device="cuda", dtype=torch.int32)
        dist = torch.empty((M, kappa), device="cuda", dtype=torch.float64)
        _check(lib().askit_query_neighbors(self.ptr, C.c_void_p(Yd.data_ptr()), M, Yd.stride(0),
                                           C.c_void_p(idx.data_ptr()), C.c_void_p(dist.data_ptr()),
                                           _stream(torch)))
        return idx, dist

    def pruning_visits(self):
        """(nodes visited per point under neighbour pruning, under distance pruning)."""
        import torch
        vk = torch.empty(self.N, device="cuda", dtype=torch.int32)
        vd = torch.empty(self.N, device="cuda", dtype=torch.int32)
        _check(lib().askit_pruning_visits(self.ptr, C.c_void_p(vk.data_ptr()), C.c_void_p(vd.data_ptr()),
                                          _stream(torch)))
        return vk, vd

    def info(self) -> dict:
        i = Info()
        _check(lib().askit_get_info(self.ptr, C.byref(i)))
        return i.as_dict()

    def export(self, item, dtype):
        n = C.c_size_t(0)
        _check(lib().askit_export(self.ptr, item, None, 0, C.byref(n)))
        dt = np.dtype(dtype)
        buf = np.empty(max(1, n.value // dt.itemsize), dtype=dt)
        _check(lib().askit_export(self.ptr, item, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                  C.byref(n)))
        return buf[: n.value // dt.itemsize]

    def close(self):
        if self.ptr:
            if getattr(self, "owned", True):
                lib().askit_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- exports
    def structures(self) -> dict:
        """Host copies of every internal structure (for verification)."""
        inf = self.info()
        nn, ell, smax, ncm = inf["num_nodes"], inf["sample_rows"], inf["max_skeleton"], inf["ncol_max"]
        kap = inf["kappa"]
        out = dict(info=inf)
        out["perm"] = self.export(X_PERM, np.int32)
        out["knn_idx"] = self.export(X_KNN_IDX, np.int32).reshape(self.N, kap)
        out["knn_d"] = self.export(X_KNN_DIST, np.float64).reshape(self.N, kap)
        out["nodes"] = self.export(X_NODES, np.uint8).view(NODE_DTYPE)
        out["nl_pos"] = self.export(X_NLIST_POS, np.int32).reshape(nn, ell)
        out["nl_key"] = self.export(X_NLIST_KEY, np.float64).reshape(nn, ell)
        out["nl_cnt"] = self.export(X_NLIST_CNT, np.int32)
        out["T"] = self.export(X_ROWS, np.int32).reshape(nn, ell)
        out["T_cnt"] = self.export(X_ROWS_CNT, np.int32)
        out["S"] = self.export(X_SKEL, np.int32).reshape(nn, smax)
        out["k"] = self.export(X_SKEL_K, np.int32)
        out["colperm"] = self.export(X_COLPERM, np.int32).reshape(nn, ncm)
        out["ncols"] = self.export(X_NCOLS, np.int32)
        out["P"] = self.export(X_PROJ, np.float32)
        out["slab_ptr"] = self.export(X_SLAB_PTR, np.int32)
        out["slab_node"] = self.export(X_SLAB_NODE, np.int32)
        out["slab_mask"] = self.export(X_SLAB_MASK, np.uint64)
        out["slab_row0"] = self.export(X_SLAB_ROW0, np.int32)
        out["hsrc"] = self.export(X_BANDWIDTH, np.float64)
        out["knn_retry"] = self.export(X_KNN_RETRY, np.int32)
        if self.nrhs:
            out["Wsk"] = self.export(X_SKEL_W, np.float32).reshape(nn, smax, self.nrhs)
        return out


def setup(X, params: Params) -> Handle:
    """Build the ASKIT structures for the points X (N x d, any array or tensor)."""
    import torch
    Xd = _dev_f32(torch, X)
    N, d = Xd.shape
    h = C.c_void_p()
    rc = lib().askit_setup(C.c_void_p(Xd.data_ptr()), N, d, Xd.stride(0), C.byref(params),
                           _stream(torch), C.byref(h))
    _check(rc)
    return Handle(h, N, d)


def knn_rptree(X, kappa, leaf_size, iterations, seed=0):
    """Approximate neighbour lists by iterated random projection trees:
    (ids N x kappa int32, squared distances N x kappa float64), device tensors."""
    import torch
    Xd = _dev_f32(torch, X)
    N, d = Xd.shape
    idx = torch.empty((N, kappa), device="cuda", dtype=torch.int32)
    dist = torch.empty((N, kappa), device="cuda", dtype=torch.float64)
    _check(lib().askit_knn_rptree(C.c_void_p(Xd.data_ptr()), N, d, Xd.stride(0), kappa, leaf_size, iterations,
                                  C.c_uint64(seed & (2**64 - 1)), C.c_void_p(idx.data_ptr()),
                                  C.c_void_p(dist.data_ptr()), _stream(torch)))
    return idx, dist


def setup_with_knn(X, knn, params: Params) -> Handle:
    """askit_setup with given neighbour lists (N x kappa original ids)."""
    import torch
    Xd = _dev_f32(torch, X)
    N, d = Xd.shape
    K = knn if torch.is_tensor(knn) else torch.from_numpy(np.ascontiguousarray(knn, dtype=np.int32))
    K = K.to(device="cuda", dtype=torch.int32).contiguous()
    assert K.shape[0] == N
    h = C.c_void_p()
    rc = lib().askit_setup_with_knn(C.c_void_p(Xd.data_ptr()), N, d, Xd.stride(0), C.c_void_p(K.data_ptr()),
                                    K.stride(0), C.byref(params), _stream(torch), C.byref(h))
    _check(rc)
    return Handle(h, N, d)


# ----------------------------------------------------------------- serving
class ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("workers", C.c_int32), ("max_batch_rhs", C.c_int32),
                ("max_batch_queries", C.c_int32), ("mem_budget", C.c_uint64), ("weight_passes", C.c_int32),
                ("max_pending", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("deferred", C.c_int64), ("batches", C.c_int64), ("batched_requests", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("p50_weights_ms", C.c_double), ("p99_weights_ms", C.c_double),
                ("p50_query_ms", C.c_double), ("p99_query_ms", C.c_double),
                ("targets_rhs", C.c_double), ("busy_s", C.c_double), ("peak_mem", C.c_uint64),
                ("joined_mid_cycle", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


SERVER_EXPORTED = ["askit_server_config_default", "askit_server_create", "askit_server_submit_weights",
                   "askit_server_submit_query", "askit_server_poll", "askit_server_wait",
                   "askit_server_stats", "askit_server_destroy"]
EXPORTED += SERVER_EXPORTED


def _server_lib():
    L = lib()
    if not getattr(L, "_server_ready", False):
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.askit_server_config_default.argtypes = [C.POINTER(ServerConfig)]
        L.askit_server_create.argtypes = [P, P, i64, i32, C.POINTER(ServerConfig), C.POINTER(P)]
        L.askit_server_submit_weights.argtypes = [P, P, i64, i32, P, i64, C.POINTER(C.c_uint64)]
        L.askit_server_submit_query.argtypes = [P, P, i64, i64, P, i64, C.POINTER(C.c_uint64)]
        L.askit_server_poll.argtypes = [P, C.c_uint64, C.POINTER(i32)]
        L.askit_server_wait.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(i32)]
        L.askit_server_stats.argtypes = [P, C.POINTER(ServerStats)]
        L.askit_server_destroy.argtypes = [P]
        L.askit_server_destroy.restype = None
        for f in SERVER_EXPORTED[:-1]:
            getattr(L, f).restype = C.c_int
        L._server_ready = True
    return L


def server_config(**kw) -> ServerConfig:
    c = ServerConfig()
    _check(_server_lib().askit_server_config_default(C.byref(c)))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _input_ready(torch):
    """Waits for the work queued so far on the caller's stream (which wrote
    the request's input), and for nothing else: a stream synchronisation of
    the legacy default stream would also wait for the server's own streams."""
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream())
    ev.synchronize()


class Server:
    """Continuous-batching server over a set-up handle (see include/askit.h).
    Device tensors passed to submit_* must stay alive until the request is done;
    the server keeps references to them until then."""

    def __init__(self, handle: Handle, W0, cfg: ServerConfig | None = None):
        import torch
        self.h = handle
        self.W0 = _dev_f32(torch, W0)
        self.nrhs0 = self.W0.shape[1]
        cfg = cfg or server_config()
        p = C.c_void_p()
        _check(_server_lib().askit_server_create(handle.ptr, C.c_void_p(self.W0.data_ptr()),
                                                 self.W0.stride(0), self.nrhs0, C.byref(cfg), C.byref(p)))
        self.ptr = p
        self._keep = {}

    def submit_weights(self, W, out=None):
        import torch
        Wd = _dev_f32(torch, W)
        U = out if out is not None else torch.empty_like(Wd)
        _input_ready(torch)   # the server reads W on its own streams
        t = C.c_uint64()
        _check(_server_lib().askit_server_submit_weights(self.ptr, C.c_void_p(Wd.data_ptr()), Wd.stride(0),
                                                         Wd.shape[1], C.c_void_p(U.data_ptr()), U.stride(0),
                                                         C.byref(t)))
        self._keep[t.value] = (Wd, U)
        return t.value

    def submit_query(self, Y, out=None):
        import torch
        Yd = _dev_f32(torch, Y)
        U = out if out is not None else torch.empty((Yd.shape[0], self.nrhs0), device="cuda",
                                                     dtype=torch.float32)
        _input_ready(torch)
        t = C.c_uint64()
        _check(_server_lib().askit_server_submit_query(self.ptr, C.c_void_p(Yd.data_ptr()), Yd.shape[0],
                                                       Yd.stride(0), C.c_void_p(U.data_ptr()), U.stride(0),
                                                       C.byref(t)))
        self._keep[t.value] = (Yd, U)
        return t.value

    def poll(self, ticket) -> int:
        st = C.c_int32()
        _check(_server_lib().askit_server_poll(self.ptr, ticket, C.byref(st)))
        return st.value

    def wait(self, ticket, timeout_s=-1.0):
        """Returns the output tensor of a finished request (raises if it failed)."""
        st = C.c_int32()
        _check(_server_lib().askit_server_wait(self.ptr, ticket, timeout_s, C.byref(st)))
        if st.value < 0:
            raise AskitError(ERR_DEVICE, lib().askit_last_error().decode())
        if st.value == 0:
            raise TimeoutError(f"request {ticket} still pending")
        return self._keep.pop(ticket)[1]

    def stats(self) -> dict:
        s = ServerStats()
        _check(_server_lib().askit_server_stats(self.ptr, C.byref(s)))
        return s.as_dict()

    def close(self):
        if self.ptr:
            _server_lib().askit_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- batched form
class BatchInfo(C.Structure):
    _fields_ = [("count", C.c_int32), ("nrhs", C.c_int32), ("total_points", C.c_int64),
                ("total_chunks", C.c_int64), ("near_entries", C.c_int64), ("far_entries", C.c_int64),
                ("near_pairs", C.c_int64), ("far_pairs", C.c_int64), ("t_setup_ms", C.c_double),
                ("t_skel_ms", C.c_double), ("tuned", C.c_int32), ("launch_blocks", C.c_int32), ("launch_plan", C.c_int32),
                ("reserved", C.c_int32), ("candidate_ms", C.c_double * 8), ("graphs", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["candidate_ms"] = list(self.candidate_ms)
        return d


BATCH_EXPORTED = ["askit_batch_setup", "askit_batch_update_weights", "askit_batch_evaluate", "askit_batch_run",
                  "askit_batch_get_info", "askit_batch_instance", "askit_batch_destroy",
                  "askit_batch_set_launch"]
EXPORTED += BATCH_EXPORTED


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.askit_batch_setup.argtypes = [i32, P, P, P, P, C.POINTER(Params), P, C.POINTER(P)]
        L.askit_batch_update_weights.argtypes = [P, P, i64, i32, P]
        L.askit_batch_evaluate.argtypes = [P, P, i64, P]
        L.askit_batch_run.argtypes = [P, P, i64, i32, P, i64, P]
        L.askit_batch_get_info.argtypes = [P, C.POINTER(BatchInfo)]
        L.askit_batch_set_launch.argtypes = [P, i32, i32, i32]
        L.askit_batch_instance.argtypes = [P, i32]
        L.askit_batch_instance.restype = P
        L.askit_batch_destroy.argtypes = [P]
        L.askit_batch_destroy.restype = None
        for f in ("askit_batch_setup", "askit_batch_update_weights", "askit_batch_evaluate", "askit_batch_run",
                  "askit_batch_get_info", "askit_batch_set_launch"):
            getattr(L, f).restype = C.c_int
        L._batch_ready = True
    return L


class Batch:
    """Many independent problems behind one handle (see include/askit.h).
    W and U stack the instances' rows in order (instance i from offsets[i])."""

    def __init__(self, Xs, params: Params):
        import torch
        ts = [_dev_f32(torch, X) for X in Xs]
        n = len(ts)
        ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        Ns = (C.c_int64 * n)(*[t.shape[0] for t in ts])
        ds = (C.c_int32 * n)(*[t.shape[1] for t in ts])
        lds = (C.c_int64 * n)(*[t.stride(0) for t in ts])
        p = C.c_void_p()
        _check(_batch_lib().askit_batch_setup(n, ptrs, Ns, ds, lds, C.byref(params), _stream(torch),
                                              C.byref(p)))
        self.ptr = p
        self.sizes = [t.shape[0] for t in ts]
        self.dims = [t.shape[1] for t in ts]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.rows = int(self.offsets[-1])
        self.nrhs = 0

    def update_weights(self, W):
        import torch
        Wd = _dev_f32(torch, W)
        assert Wd.shape[0] == self.rows
        _check(_batch_lib().askit_batch_update_weights(self.ptr, C.c_void_p(Wd.data_ptr()), Wd.stride(0),
                                                       Wd.shape[1], _stream(torch)))
        self.nrhs = Wd.shape[1]

    def evaluate(self, out=None):
        import torch
        U = out if out is not None else torch.empty((self.rows, self.nrhs), device="cuda", dtype=torch.float32)
        _check(_batch_lib().askit_batch_evaluate(self.ptr, C.c_void_p(U.data_ptr()), U.stride(0),
                                                 _stream(torch)))
        return U

    def run(self, W, out):
        """update_weights + evaluate through the cached graph; W and out are
        device tensors that must stay allocated while the batch may replay them."""
        import torch
        assert torch.is_tensor(W) and W.is_cuda and W.dtype == torch.float32 and W.shape[0] == self.rows
        _check(_batch_lib().askit_batch_run(self.ptr, C.c_void_p(W.data_ptr()), W.stride(0), W.shape[1],
                                            C.c_void_p(out.data_ptr()), out.stride(0), _stream(torch)))
        self.nrhs = W.shape[1]
        return out

    def set_launch(self, nrhs, blocks, plan=0):
        _check(_batch_lib().askit_batch_set_launch(self.ptr, nrhs, blocks, plan))

    def info(self) -> dict:
        i = BatchInfo()
        _check(_batch_lib().askit_batch_get_info(self.ptr, C.byref(i)))
        return i.as_dict()

    def instance(self, i) -> Handle:
        hp = _batch_lib().askit_batch_instance(self.ptr, i)
        if not hp:
            raise IndexError(i)
        h = Handle(C.c_void_p(hp), self.sizes[i], self.dims[i])
        h.owned = False
        return h

    def close(self):
        if self.ptr:
            _batch_lib().askit_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
