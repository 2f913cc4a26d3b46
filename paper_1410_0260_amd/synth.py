"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only: point clouds, weight vectors,
query batches and request streams.  It holds none of the method's
arithmetic, so both the FP64 oracle (tests) and the HIP path (binding,
bench) may draw their inputs from it.

The paper's experiments use normal point clouds of low intrinsic
dimension embedded in a higher ambient dimension (Sec. 4, "Synthetic
datasets"; runs 27-28 embed 4-D data in 1000-D).  The generator below
draws a Gaussian mixture on a random q-dimensional subspace of R^d
(random orthogonal embedding) and adds isotropic ambient noise whose
variance is `noise_var`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class Workload:
    """One problem instance: generator recipe plus method parameters."""

    name: str
    N: int
    d: int
    q: int                 # intrinsic dimension of the mixture
    n_comp: int            # mixture components (equal weights)
    noise_var: float       # variance of the ambient N(0, noise_var) noise
    h: float               # Gaussian bandwidth, K = exp(-r^2 / (2 h^2)); 0 => variable
    m: int                 # leaf size
    kappa: int             # nearest neighbours per point
    smax: int              # maximum skeleton size
    ell: int               # sampled rows per node (0 => smax + 20)
    tau: float             # ID tolerance relative to |R_00|
    R: int                 # right-hand sides
    seed: int
    bw_neighbor: int = 0   # variable bandwidth: h_j = distance to this neighbour (1-based)
    spread: float = 3.0    # component means ~ spread * N(0, I_q)
    prune_levels: int = 0  # > 0: only the prune_levels deepest tree levels may be pruned
    extra: dict = field(default_factory=dict)

    @property
    def ell_eff(self) -> int:
        return self.ell if self.ell > 0 else self.smax + 20

    def as_dict(self) -> dict:
        return asdict(self)


def mixture_points(N: int, d: int, q: int, n_comp: int, noise_var: float, seed: int,
                   spread: float = 3.0, basis_seed: int | None = None,
                   rng: np.random.Generator | None = None) -> np.ndarray:
    """Gaussian mixture on a random q-dim subspace of R^d plus ambient noise (FP32).

    The subspace basis Q and the component means depend only on
    `basis_seed` (default: `seed`), so query batches can be drawn from the
    same distribution as a resident point set.
    """
    bseed = seed if basis_seed is None else basis_seed
    brng = np.random.default_rng(bseed)
    A = brng.standard_normal((d, q))
    Qm, Rm = np.linalg.qr(A)
    Qm = Qm * np.sign(np.diag(Rm))[None, :]
    mu = spread * brng.standard_normal((n_comp, q))
    g = np.random.default_rng(seed) if rng is None else rng
    comp = g.integers(n_comp, size=N)
    z = mu[comp] + g.standard_normal((N, q))
    X = np.empty((N, d), dtype=np.float32)
    chunk = 1 << 16
    sd = math.sqrt(noise_var)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        X[a:b] = (z[a:b] @ Qm.T + sd * g.standard_normal((b - a, d))).astype(np.float32)
    return X


# ---------------------------------------------------------------------------
# Point sets of the pruning comparison (Table t:prune).
# ---------------------------------------------------------------------------

def curve_points(N: int, d: int, seed: int) -> np.ndarray:
    """The paper's curve: x_i = f(i pi t), t uniform in [0, 1], i = 1..d, f = cos
    for odd i and sin for even i (intrinsic dimension one)."""
    t = np.random.default_rng(seed).random(N)
    i = np.arange(1, d + 1)
    arg = np.pi * t[:, None] * i[None, :]
    return np.where(i % 2 == 1, np.cos(arg), np.sin(arg)).astype(np.float32)


def gaussian_points(N: int, d: int, seed: int) -> np.ndarray:
    """Standard normal points in d dimensions (intrinsic dimension d)."""
    return np.random.default_rng(seed).standard_normal((N, d)).astype(np.float32)


def sphere_points(N: int, d: int, seed: int) -> np.ndarray:
    """Points uniform on the unit sphere S^4 of a random 5-dim subspace
    (intrinsic dimension four) for d >= 5; for d = 4, uniform on S^3."""
    g = np.random.default_rng(seed)
    k = 5 if d >= 5 else d
    z = g.standard_normal((N, k))
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    if k == d:
        return z.astype(np.float32)
    Q, Rm = np.linalg.qr(g.standard_normal((d, k)))
    Q = Q * np.sign(np.diag(Rm))[None, :]
    return (z @ Q.T).astype(np.float32)


def weights(N: int, R: int, seed: int) -> np.ndarray:
    """Weights w ~ N(0, 1), FP32, N x R row-major."""
    g = np.random.default_rng(seed + 7919)
    return g.standard_normal((N, R), dtype=np.float32)


def points(w: Workload) -> np.ndarray:
    return mixture_points(w.N, w.d, w.q, w.n_comp, w.noise_var, w.seed, w.spread)


def queries(w: Workload, M: int, seed: int) -> np.ndarray:
    """Query points from the same mixture as `points(w)` (same basis and means)."""
    return mixture_points(M, w.d, w.q, w.n_comp, w.noise_var, seed, w.spread, basis_seed=w.seed)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the paper's experiments in shape (Sec. 4):
# low intrinsic dimension in a larger ambient space, leaf sizes of a few
# hundred points, skeletons of up to a few hundred points, l = s + 20.
# ---------------------------------------------------------------------------

def small_fp64() -> Workload:
    """4096 points in 8-D, 3-dim intrinsic, 4 components; fully checkable on the CPU."""
    return Workload("gauss-mix N=4096 d=8 m=128 k=16 s=64", N=4096, d=8, q=3, n_comp=4,
                    noise_var=1e-3, h=0.5, m=128, kappa=16, smax=64, ell=84, tau=1e-6,
                    R=1, seed=1)


def fp32_1m() -> Workload:
    """2^20 points in 64-D, 8-dim intrinsic, 16 components."""
    return Workload("gauss-mix N=1048576 d=64 m=512 k=32 s=256", N=1 << 20, d=64, q=8,
                    n_comp=16, noise_var=1e-3, h=1.0, m=512, kappa=32, smax=256, ell=276,
                    tau=1e-5, R=1, seed=2)


def fp32_1m_gate() -> Workload:
    """The 2^20-point, 64-D workload with a wide kernel (h = 16), every other
    parameter as listed.  At the listed h = 1 the approximation's own error
    with s <= 256 is about 0.27; with h = 16 the far field carries nearly all
    of u (the near-field part alone is off by 99%) and the method is within
    the 1e-3 accuracy target."""
    return Workload("gauss-mix N=1048576 d=64 m=512 k=32 s=256 h=16", N=1 << 20, d=64, q=8,
                    n_comp=16, noise_var=1e-3, h=16.0, m=512, kappa=32, smax=256, ell=276,
                    tau=1e-5, R=1, seed=2)


def mixed_1000d() -> Workload:
    """2^18 points in 1000-D, 6-dim intrinsic, 8 components, 16 right-hand sides."""
    return Workload("gauss-mix N=262144 d=1000 m=512 k=32 s=256 R=16", N=1 << 18, d=1000, q=6,
                    n_comp=8, noise_var=1e-4, h=2.0, m=512, kappa=32, smax=256, ell=276,
                    tau=1e-5, R=16, seed=3)


def serving_4m() -> Workload:
    """2^22 resident points in 64-D, 8-dim intrinsic, 32 components."""
    return Workload("gauss-mix N=4194304 d=64 m=512 k=32 s=256", N=1 << 22, d=64, q=8,
                    n_comp=32, noise_var=1e-3, h=1.0, m=512, kappa=32, smax=256, ell=276,
                    tau=1e-5, R=1, seed=5)


def batched_instances(count: int = 256, seed: int = 4000) -> list[Workload]:
    """Uneven independent problems: N log-uniform in [2048, 65536], d in {16, 32, 64},
    4-dim intrinsic, variable bandwidth h_j = distance to the 16th neighbour."""
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        N = int(round(math.exp(g.uniform(math.log(2048), math.log(65536)))))
        d = int(g.choice([16, 32, 64]))
        out.append(Workload(f"inst{k} N={N} d={d}", N=N, d=d, q=4, n_comp=1, noise_var=1e-3,
                            h=0.0, m=256, kappa=16, smax=128, ell=148, tau=1e-5, R=1,
                            seed=seed + k, bw_neighbor=16))
    return out


def request_stream(duration_s: float, rate_hz: float, seed: int = 55,
                   max_rhs: int = 64, max_queries: int = 4096) -> list[dict]:
    """Poisson arrivals; half weight-vector requests (R ~ U{1..max_rhs}), half
    query batches (M = round(exp U[0, ln max_queries]))."""
    g = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += g.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        if g.random() < 0.5:
            out.append({"t": t, "kind": "weights", "R": int(g.integers(1, max_rhs + 1)),
                        "seed": int(g.integers(1 << 31))})
        else:
            M = int(round(math.exp(g.uniform(0.0, math.log(max_queries)))))
            out.append({"t": t, "kind": "query", "M": max(1, M), "seed": int(g.integers(1 << 31))})
    return out
