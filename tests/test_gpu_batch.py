"""Batched form: a batch of uneven instances (different N, none a power of
two, different d, variable bandwidth) gives, for every instance, the u that
the single-problem calls give for it alone -- bit for bit, in every launch
shape of the fused evaluation -- and the FP64 oracle's u within the parity
tolerance; the captured graph gives the eager result on every replay, with
other device work and new weight values between replays."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_0260_amd import synth
from tests.gpu_common import rel

pytestmark = pytest.mark.gpu

SIZES = [(700, 8), (2999, 16), (1234, 40), (300, 8), (2048, 16), (1801, 24), (555, 40), (4000, 8)]
P = O.Params(m=64, kappa=16, smax=32, ell=52, tau=1e-5, h=0.0, bw_neighbor=8, seed=21)


def _gparams():
    from paper_1410_0260_amd import askit as A
    return A.default_params(leaf_size=P.m, kappa=P.kappa, max_skeleton=P.smax, sample_rows=P.ell, id_tol=P.tau,
                            bandwidth=1.0, bw_neighbor=P.bw_neighbor, seed=P.seed)


@pytest.fixture(scope="module")
def batch():
    import torch
    from paper_1410_0260_amd import askit as A
    Xs = [synth.mixture_points(n, d, 4, 1, 1e-3, 500 + i) for i, (n, d) in enumerate(SIZES)]
    print(f"\n[batch] {len(Xs)} instances, sizes {SIZES}", flush=True)
    b = A.Batch([torch.from_numpy(X).cuda() for X in Xs], _gparams())
    yield A, b, Xs
    b.close()


def _alone(A, Xs, W, offsets):
    import torch
    out = []
    for i, X in enumerate(Xs):
        h = A.setup(torch.from_numpy(X).cuda(), _gparams())
        h.update_weights(torch.from_numpy(np.ascontiguousarray(W[offsets[i]:offsets[i + 1]])).cuda())
        out.append(h.evaluate().cpu().numpy())
        h.close()
    return out


@pytest.mark.parametrize("R", [1, 3, 9, 40])
def test_every_launch_shape_equals_alone(batch, R):
    """Every grid form and column-tile plan (wide: 64/32-column MFMA passes
    and 4/1-column vector passes; narrow: 32 and 1) gives each instance's
    u bit for bit as set up and evaluated alone."""
    import torch
    A, b, Xs = batch
    W = synth.weights(b.rows, R, 77 + R)
    alone = _alone(A, Xs, W, b.offsets)
    b.update_weights(torch.from_numpy(W).cuda())
    for plan in (0, 1):
        for blocks in (0, 256, 1024, 3):
            b.set_launch(R, blocks, plan)
            U = b.evaluate().cpu().numpy()
            for i in range(len(Xs)):
                assert np.array_equal(U[b.offsets[i]:b.offsets[i + 1]], alone[i]), \
                    f"plan {plan} blocks {blocks} instance {i}"


def test_matches_oracle(batch):
    import torch
    A, b, Xs = batch
    W = synth.weights(b.rows, 2, 5)
    b.update_weights(torch.from_numpy(W).cuda())
    b.set_launch(2, 0)
    U = b.evaluate().cpu().numpy().astype(np.float64)
    for i in (0, 2, 3):
        Wi = np.ascontiguousarray(W[b.offsets[i]:b.offsets[i + 1]])
        st = O.run_askit(Xs[i], Wi, P, record=False)
        for r in range(2):
            assert rel(U[b.offsets[i]:b.offsets[i + 1], r], st["ev"].U[:, r]) < 1e-5, f"instance {i}"


def test_graph_replays_equal_eager(batch):
    import torch
    A, b, Xs = batch
    R = 4
    Ws = [synth.weights(b.rows, R, 900 + k) for k in range(3)]
    ref = []
    for W in Ws:
        b.update_weights(torch.from_numpy(W).cuda())
        ref.append(b.evaluate().cpu().numpy())
    Wd = torch.empty((b.rows, R), device="cuda", dtype=torch.float32)
    Ud = torch.empty((b.rows, R), device="cuda", dtype=torch.float32)
    other = torch.empty((b.rows, R), device="cuda", dtype=torch.float32)
    for rep in range(6):
        k = rep % 3
        Wd.copy_(torch.from_numpy(Ws[k]))
        Ud.fill_(float("nan"))
        b.run(Wd, Ud)
        torch.cuda.synchronize()
        assert np.array_equal(Ud.cpu().numpy(), ref[k]), f"replay {rep}"
        # eager work of the program between replays
        b.update_weights(torch.from_numpy(Ws[(k + 1) % 3]).cuda())
        b.evaluate(out=other)
        torch.cuda.synchronize()
        assert np.array_equal(other.cpu().numpy(), ref[(k + 1) % 3])
    inf = b.info()
    assert inf["tuned"] == 1 and inf["graphs"] == 1
    assert inf["launch_blocks"] in (0, 2 * 256, 4 * 256, 8 * 256) or inf["launch_blocks"] % 256 == 0
    assert inf["launch_plan"] in (0, 1)
    assert all(t > 0 for t in inf["candidate_ms"])
