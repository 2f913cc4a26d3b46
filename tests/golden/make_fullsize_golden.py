"""Expected values of the full-size parity test, written by the FP64 oracle alone.

Runs the whole oracle pipeline (Alg. 5: exact neighbours, tree, node lists
(Alg. 2), sampled rows (Eq. e:sk_targets), skeletonization (Alg. 3),
skeleton weights, then Alg. 4) on the 2^20-point, 64-dimensional workload
and stores what the GPU test compares:

  * u at 10,000 seeded targets (the paper measures the error on 10K sampled
    targets, Sec. 3), the near-field part of u at the same targets (the
    paper's eps_kappa), and the FP64 direct sum u_dir there (Eq. e:problem);
  * per target, the number of near leaves and pruned nodes of its Alg. 4
    traversal and two sums over their ids (an exact fingerprint of the
    interaction lists);
  * about 200 seeded nodes across every level: rank k, skeleton (tree
    positions) and the oracle's decision margins;
  * 8 of them (leaves and internal nodes of several levels): the column
    order of the ID, P applied to four seeded vectors, the Frobenius norm of
    P, and the skeleton weights.

Only `oracle/` and the input generators are used; nothing here touches the
HIP library.  The neighbour lists (the costly stage: N^2 d FP64 products)
are cached in --cache so that other bandwidths reuse them (they do not depend
on h).

Usage: python tests/golden/make_fullsize_golden.py --h 1.0 [--threads 6]
       [--cache /tmp/askit_fullsize_cache]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

TARGET_SEED = 20141001
NODE_SEED = 20141002
SKETCH_SEED = 20141003
N_TARGETS = 10000
SKETCH_COLS = 4


def golden_name(h: float) -> str:
    return os.path.join(HERE, f"fullsize_fp32_1m_h{h:g}.npz")


def pick_targets(N):
    import numpy as np
    return np.sort(np.random.default_rng(TARGET_SEED).choice(N, N_TARGETS, replace=False))


def pick_nodes(nodes):
    """Every node of levels 1-4 and 24 seeded nodes of each deeper level; the
    8 P nodes: two leaves and one node of levels 9, 7, 5, 3, 2, 1."""
    import numpy as np
    rng = np.random.default_rng(NODE_SEED)
    lev = nodes["level"]
    out = []
    for L in range(1, int(lev.max()) + 1):
        ids = np.nonzero(lev == L)[0]
        out.extend(ids if len(ids) <= 24 else np.sort(rng.choice(ids, 24, replace=False)))
    out = np.array(out, dtype=np.int64)
    leaves = [a for a in out if nodes[a]["left"] < 0]
    pn = list(rng.choice(leaves, 2, replace=False))
    for L in (9, 7, 5, 3, 2, 1):
        c = [a for a in out if lev[a] == L and nodes[a]["left"] >= 0]
        if c:
            pn.append(int(rng.choice(c)))
    return out, np.array(pn[:8], dtype=np.int64)


def sketch_vectors(ncol_max):
    import numpy as np
    return np.random.default_rng(SKETCH_SEED).standard_normal((ncol_max, SKETCH_COLS))


def list_fingerprint(ids_per_target):
    import numpy as np
    cnt = np.array([len(a) for a in ids_per_target], np.int64)
    s1 = np.array([int(np.sum(a.astype(np.int64))) for a in ids_per_target], np.int64)
    s2 = np.array([int(np.sum(a.astype(np.int64) ** 2)) for a in ids_per_target], np.int64)
    return cnt, s1, s2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=float, action="append", required=True)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--cache", default="/tmp/askit_fullsize_cache")
    ap.add_argument("--n", type=int, default=0, help="trial run on the first n points (output in --cache)")
    args = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = str(args.threads)
    import dataclasses

    import numpy as np

    from oracle import oracle as O
    from paper_1410_0260_amd import synth

    base = synth.fp32_1m()
    if args.n:
        base = dataclasses.replace(base, N=args.n)
    X = synth.points(base)
    W = synth.weights(base.N, base.R, base.seed)
    N = base.N
    os.makedirs(args.cache, exist_ok=True)
    kpath = os.path.join(args.cache, f"knn_{N}_{base.d}_{base.kappa}_{base.seed}.npz")
    t0 = time.time()
    if os.path.exists(kpath):
        z = np.load(kpath)
        kidx, kd = z["idx"], z["dist"]
        t_knn = float(z["seconds"])
        print(f"[golden] neighbour lists from {kpath}", flush=True)
    else:
        print(f"[golden] exhaustive kNN of {N} points on {args.threads} threads", flush=True)
        kidx, kd = O.knn(X, X, base.kappa, exclude_self=True)
        t_knn = time.time() - t0
        np.savez(kpath, idx=kidx, dist=kd, seconds=t_knn)
        print(f"[golden] kNN {t_knn:.0f} s", flush=True)
    tg = pick_targets(N) if N > N_TARGETS else np.arange(N)
    t1 = time.time()
    Ud = O.direct(X[tg], X, W, base.h if base.h > 0 else 1.0)
    t_direct = time.time() - t1
    print(f"[golden] FP64 direct sum at {len(tg)} targets: {t_direct:.0f} s", flush=True)
    for h in args.h:
        wl = dataclasses.replace(base, h=h)
        p = O.Params.from_workload(wl)
        t2 = time.time()
        st = O.setup(X, p, knn_lists=(kidx, kd))
        t_setup = time.time() - t2
        print(f"[golden] h={h}: tree, lists, rows, skeletons {t_setup:.0f} s", flush=True)
        Wtree = W[st["perm"]].astype(np.float64)
        Wsk = O.upward(st["nodes"], Wtree, st["sk"], p.smax)
        nb = O.self_neighbours(st, tg)
        t3 = time.time()
        ev = O.evaluate(X[tg], nb, X, st["perm"], st["nodes"], None, p.h, W, st["sk"], Wsk, p.smax,
                        record=True)
        t_eval = time.time() - t3
        ud = Ud if h == base.h else O.direct(X[tg], X, W, h)
        eps = float(np.linalg.norm(ev.U[:, 0] - ud[:, 0]) / np.linalg.norm(ud[:, 0]))
        eps_near = float(np.linalg.norm(ev.Unear[:, 0] - ud[:, 0]) / np.linalg.norm(ud[:, 0]))
        print(f"[golden] h={h}: eps {eps:.3e}, near-only eps {eps_near:.3e}", flush=True)
        nodes, sk = st["nodes"], st["sk"]
        samp, pn = pick_nodes(nodes)
        V = sketch_vectors(sk.ncol_max)
        pc = np.full((len(pn), sk.ncol_max), -1, np.int32)
        psk = np.zeros((len(pn), p.smax, SKETCH_COLS))
        pfro = np.zeros(len(pn))
        wsk = np.zeros((len(pn), p.smax))
        for r, a in enumerate(pn):
            k, n = int(sk.k[a]), int(sk.ncols[a])
            Pa = sk.proj(a)
            pc[r, :n] = sk.colperm[a, :n]
            psk[r, :k] = Pa @ V[:n - k]
            pfro[r] = np.linalg.norm(Pa)
            wsk[r, :k] = Wsk[a, :k, 0]
        ncnt, ns1, ns2 = list_fingerprint(ev.near)
        fcnt, fs1, fs2 = list_fingerprint(ev.far)
        near_leaf_pts = np.array([int(np.sum(nodes["hi"][a] - nodes["lo"][a])) for a in ev.near], np.int64)
        far_skel_pts = np.array([int(np.sum(sk.k[a])) for a in ev.far], np.int64)
        out = golden_name(h) if not args.n else os.path.join(args.cache, f"trial_{N}_h{h:g}.npz")
        np.savez_compressed(
            out, targets=tg, u=ev.U[:, 0], u_near=ev.Unear[:, 0], u_direct=ud[:, 0],
            near_cnt=ncnt, near_s1=ns1, near_s2=ns2, far_cnt=fcnt, far_s1=fs1, far_s2=fs2,
            near_points=near_leaf_pts, far_points=far_skel_pts,
            nodes=samp, k=sk.k[samp], S=sk.S[samp], piv_margin=sk.piv_margin[samp],
            rank_margin=sk.rank_margin[samp], p_nodes=pn, p_colperm=pc, p_ncols=sk.ncols[pn],
            p_sketch=psk, p_fro=pfro, wsk=wsk, eps=eps, eps_near=eps_near, h=h)
        summary = {
            "workload": wl.name, "h": h, "N": N, "d": wl.d, "m": wl.m, "kappa": wl.kappa, "s_max": wl.smax,
            "l": wl.ell_eff, "tau": wl.tau, "targets": len(tg), "eps": eps, "eps_near": eps_near,
            "rank_cap_nodes": int(np.sum(sk.k[1:] == p.smax)), "nodes": int(len(nodes) - 1),
            "mean_near_leaves": float(ncnt.mean()), "mean_far_nodes": float(fcnt.mean()),
            "seconds": {"knn": t_knn, "direct": t_direct, "setup_rest": t_setup, "evaluate": t_eval},
            "threads": args.threads, "cpu": platform.processor() or platform.machine(),
        }
        with open(out.replace(".npz", ".json"), "w") as f:
            json.dump(summary, f, indent=1)
        print(f"[golden] wrote {out}: {json.dumps(summary)}", flush=True)
        del st, sk, Wsk, ev


if __name__ == "__main__":
    main()
