"""Shared helpers of the GPU parity tests: run the oracle and the HIP path on
the same seeded inputs and expand the library's slab interaction lists."""
import numpy as np

from oracle import oracle as O


def run_both(X, W, wl_params, gpu_params, Y=None):
    import torch
    from paper_1410_0260_amd import askit as A
    st = O.run_askit(X, W, wl_params, record=True)
    h = A.setup(torch.from_numpy(X).cuda(), gpu_params)
    h.update_weights(torch.from_numpy(W).cuda())
    U = h.evaluate()
    torch.cuda.synchronize()
    g = h.structures()
    g["U"] = U.cpu().numpy().astype(np.float64)
    if Y is not None:
        g["Y"] = Y
        Uq = h.query(torch.from_numpy(Y).cuda())
        torch.cuda.synchronize()
        g["Uq"] = Uq.cpu().numpy().astype(np.float64)
        qi, qd = h.query_neighbors(torch.from_numpy(Y).cuda())
        g["qidx"], g["qd"] = qi.cpu().numpy(), qd.cpu().numpy()
        st["query"] = O.query(st, Y)
    h.close()
    return st, g


def slab_lists(g, N):
    """Per tree position: (sorted near node ids, sorted far node ids)."""
    ptr, node, mask, row0 = g["slab_ptr"], g["slab_node"], g["slab_mask"], g["slab_row0"]
    ns = len(row0)
    near = [[] for _ in range(N)]
    far = [[] for _ in range(N)]
    for s in range(ns):
        for lo, hi, out in ((ptr[s], ptr[s + 1], near), (ptr[ns + 1 + s], ptr[ns + 2 + s], far)):
            for e in range(lo, hi):
                m = int(mask[e])
                b = 0
                while m:
                    if m & 1:
                        out[row0[s] + b].append(int(node[e]))
                    m >>= 1
                    b += 1
    return [sorted(a) for a in near], [sorted(a) for a in far]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
