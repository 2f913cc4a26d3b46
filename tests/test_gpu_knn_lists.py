"""Tile lists of the kNN filter sweeps against the unlisted sweeps on the
2^20-point, 64-D workload (needs an MI355X).

The lists skip only (row group, tile) pairs that cannot hold a survivor, so
each row's survivor count is the same with and without them: the same rows
overflow their slots, and the neighbour lists (exact either way) agree.
ASKIT_KNN_NO_SKIP=1 makes both the symmetric sweep and the overflowed rows'
sweep visit every pair."""
import os

import numpy as np
import pytest

from paper_1410_0260_amd import synth

pytestmark = pytest.mark.gpu


def _setup(X, prm, lists):
    import torch
    from paper_1410_0260_amd import askit as A
    if lists:
        os.environ.pop("ASKIT_KNN_NO_SKIP", None)
    else:
        os.environ["ASKIT_KNN_NO_SKIP"] = "1"
    try:
        h = A.setup(torch.from_numpy(X).cuda(), prm)
        torch.cuda.synchronize()
        inf = h.info()
        idx = h.export(A.X_KNN_IDX, np.int32)
        dist = h.export(A.X_KNN_DIST, np.float64)
        h.close()
    finally:
        os.environ.pop("ASKIT_KNN_NO_SKIP", None)
    return inf, idx, dist


def test_tile_lists_keep_every_survivor():
    from paper_1410_0260_amd import askit as A
    wl = synth.fp32_1m_gate()
    X = synth.points(wl)
    prm = A.params_from_workload(wl)
    li, lidx, ldist = _setup(X, prm, True)
    fi, fidx, fdist = _setup(X, prm, False)
    print(f"\n[tile lists] wave tiles swept {li['knn_tiles_swept']}, overflowed rows {li['knn_retry_rows']} "
          f"(unlisted {fi['knn_retry_rows']}), uncertified {li['knn_uncertified_rows']} "
          f"(unlisted {fi['knn_uncertified_rows']})", flush=True)
    n_tiles = (wl.N + 63) // 64
    all_waves = sum(4 * (n_tiles - 2 * b) for b in range((wl.N + 127) // 128))
    assert 0 < li["knn_tiles_swept"] < all_waves
    assert fi["knn_tiles_swept"] == -1
    assert li["knn_retry_rows"] == fi["knn_retry_rows"] > 0
    assert np.array_equal(lidx, fidx)
    assert np.array_equal(ldist, fdist)
