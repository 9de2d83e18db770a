"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method (no transforms, no structure
factor, no loss): it only draws positions and lays out targets and weights on
the dense mode cube.  It is shared by the tests, the benchmark and the smoke
check, and by both sides of every parity comparison.

Mode cube layout: C order over (n_0, ..., n_{d-1}), each n_a running from -M to
M, so the entry for mode vector n sits at index (n_0 + M, ..., n_{d-1} + M).

Workloads (positions i.i.d. uniform in a periodic box, the Poisson starting
point of every minimisation in the paper; targets are the stealthy and
power-law families of the main text; the constrained region is counted in
integer mode units n, k = 2 pi n / L):
"""
from __future__ import annotations

import math

import numpy as np

WORKLOADS = {
    # small FP64 case that the direct-sum oracle finishes in well under a second
    "2d_n1024_stealthy16_f64": dict(d=2, N=1024, L=32.0, M=16, kcut=16.0, dtype="f64",
                                   tol=1e-12, target="stealthy", seed=1001),
    # the headline 2D case
    "2d_n1e6_stealthy300_f32": dict(d=2, N=1_000_000, L=1000.0, M=300, kcut=300.0,
                                   dtype="f32", tol=1e-6, target="stealthy", seed=1002),
    # the headline 3D case (plus a soft-core harmonic repulsion of diameter 0.5)
    "3d_n1e7_stealthy60_f32": dict(d=3, N=10_000_000, L=10_000_000 ** (1.0 / 3.0), M=60,
                                  kcut=60.0, dtype="f32", tol=1e-6, target="stealthy",
                                  sigma=0.5, eps=1.0, seed=1003),
    # very large 2D case
    "2d_n1e9_stealthy6000_f32": dict(d=2, N=1_000_000_000, L=31623.0, M=6000, kcut=6000.0,
                                    dtype="f32", tol=1e-5, target="stealthy", seed=1005),
}


def box_side_for_density(N: int, d: int, density: float = 1.0) -> float:
    return float((N / density) ** (1.0 / d))


def positions(N: int, d: int, L, dtype=np.float32, seed: int = 0) -> np.ndarray:
    """N points i.i.d. uniform in [0, L)^d, shape [N][d], cast to dtype."""
    rng = np.random.default_rng(seed)
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (d,))
    out = np.empty((N, d), dtype=dtype)
    chunk = 1 << 24
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        out[s:e] = rng.uniform(0.0, 1.0, (e - s, d)) * L
    # rounding of the cast may land on L itself; keep every coordinate in [0, L)
    for a in range(d):
        col = out[:, a]
        col[col >= L[a]] = 0
    return out


def mode_norm2(d: int, M: int) -> np.ndarray:
    """|n|^2 on the mode cube (integer)."""
    ax = np.arange(-M, M + 1, dtype=np.int64) ** 2
    out = ax
    for _ in range(d - 1):
        out = out[..., None] + ax
    return out


def stealthy_target(d: int, M: int, kcut: float):
    """Stealthy target: S0 = 0 with weight 1 on 0 < |n| <= kcut (inclusive).
    Returns (w, S0) cubes (float64)."""
    n2 = mode_norm2(d, M)
    w = ((n2 > 0) & (n2 <= kcut * kcut)).astype(np.float64)
    return w, np.zeros_like(w)


def power_law_target(d: int, M: int, K: float, alpha: float):
    """Power-law target S0 = (|n| / K)^alpha on 0 < |n| < K (strict), weight 1.
    Returns (w, S0) cubes (float64)."""
    n2 = mode_norm2(d, M).astype(np.float64)
    inside = (n2 > 0) & (n2 < K * K)
    w = inside.astype(np.float64)
    S0 = np.where(inside, (np.sqrt(n2) / K) ** alpha, 0.0)
    return w, S0


def ragged_batch(nb: int = 256, nmin: int = 1000, nmax: int = 100_000, kcut: int = 20,
                 alphas=(1.0, 2.0, 4.0), seed: int = 1004):
    """Ragged batch of independent 2D configurations: N_b log-uniform in [nmin, nmax],
    unit density (L_b = sqrt(N_b)), power-law targets with exponent drawn from
    `alphas` on |n| < kcut.  Returns a list of dicts (N, L, alpha, seed)."""
    rng = np.random.default_rng(seed)
    Ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nb))).astype(np.int64)
    al = rng.choice(np.asarray(alphas, dtype=np.float64), nb)
    return [dict(N=int(Ns[b]), L=math.sqrt(float(Ns[b])), alpha=float(al[b]), kcut=kcut,
                 seed=seed * 1000 + b) for b in range(nb)]


def polydisperse_strengths(N: int, d: int, seed: int = 0, ratio: float = 1.4,
                           signed: bool = False) -> np.ndarray:
    """Strengths of a 50:50 bidisperse packing of diameters 1 and `ratio`: each
    particle weighs its volume over the mean volume, c = D^d / <D^d> (float64).
    signed=True flips a random half of them (a real field of either sign)."""
    rng = np.random.default_rng(seed)
    D = np.where(rng.random(N) < 0.5, 1.0, ratio)
    v = D ** d
    c = v / v.mean()
    if signed:
        c = c * rng.choice([-1.0, 1.0], N)
    return c


def square_lattice(m: int, L: float, d: int = 2, shift=None, dtype=np.float64) -> np.ndarray:
    """m^d points on a simple cubic lattice of spacing L/m (optionally shifted)."""
    ax = (np.arange(m, dtype=np.float64) + 0.0) * (L / m)
    g = np.meshgrid(*([ax] * d), indexing="ij")
    p = np.stack([x.reshape(-1) for x in g], axis=1)
    if shift is not None:
        p = (p + np.asarray(shift, dtype=np.float64)) % L
    return p.astype(dtype)
