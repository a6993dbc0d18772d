"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws points and
strengths with numpy's PCG64 generator and records the configuration
parameters (cell, periodicity, leaf tiling, split width sigma, cutoff).

The workloads follow the point distributions the paper uses for its
experiments (Sec. 6: uniform points, and half uniform / half clustered points)
at the sizes of the residual-interaction workloads this library is measured
on.  The split width is set from the cutoff r_c = h (leaf box side) by
sigma = h / t_c, where t_c is the point at which the kernel's slowest
residual window function falls to 1e-12:

  erfc(t)                     = 1e-12 at t = 5.042030  (harmonic)
  erfc(t) + 2 t phi(t)        = 1e-12 at t = 5.427695  (Stokeslet, rotlet)
  4 t^3 phi(t)                = 1e-12 at t = 5.807081  (stresslet)

with phi(t) = exp(-t^2)/sqrt(pi).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KERNEL_IDS = {"laplace": 0, "stokeslet": 1, "stresslet": 2, "rotlet": 3}
M_IN = {"laplace": 1, "stokeslet": 3, "stresslet": 9, "rotlet": 3}
M_OUT = {"laplace": 1, "stokeslet": 3, "stresslet": 3, "rotlet": 3}

T_CUT = {"laplace": 5.042030, "stokeslet": 5.427695, "rotlet": 5.427695, "stresslet": 5.807081}


@dataclass
class Workload:
    name: str
    kernel: str
    D: int
    L: tuple
    n: tuple
    N: int
    sigma: float
    rc: float
    x: np.ndarray = field(repr=False)     # [N, 3] float64, original order
    rho: np.ndarray = field(repr=False)   # [N, m_in] float64
    seed: int = 0

    @property
    def h(self):
        return tuple(self.L[i] / self.n[i] for i in range(3))


def _uniform(rng, N, L):
    return rng.random((N, 3)) * np.asarray(L, dtype=np.float64)


def _clustered(rng, N, L, D, frac=0.7, ncl=20, std=0.02):
    """frac of the points in ncl Gaussian clusters (std per coordinate), the
    rest uniform.  Cluster points wrap in periodic axes; in free axes an
    out-of-cell coordinate is redrawn from the same cluster."""
    L = np.asarray(L, dtype=np.float64)
    nc = int(round(frac * N))
    centers = rng.random((ncl, 3)) * L
    which = rng.integers(0, ncl, size=nc)
    pts = centers[which] + rng.normal(0.0, std, size=(nc, 3))
    for ax in range(3):
        if ax < D:
            pts[:, ax] = np.mod(pts[:, ax], L[ax])
            pts[:, ax] = np.where(pts[:, ax] >= L[ax], 0.0, pts[:, ax])
        else:
            bad = (pts[:, ax] < 0.0) | (pts[:, ax] >= L[ax])
            while bad.any():
                pts[bad, ax] = centers[which[bad], ax] + rng.normal(0.0, std, size=int(bad.sum()))
                bad = (pts[:, ax] < 0.0) | (pts[:, ax] >= L[ax])
    uni = _uniform(rng, N - nc, L)
    allp = np.concatenate([pts, uni], axis=0)
    return allp[rng.permutation(N)]


def _strengths(rng, kernel, N, neutral_charges=False, zero_mean=True):
    if kernel == "laplace":
        if neutral_charges:
            q = np.concatenate([np.ones(N // 2), -np.ones(N - N // 2)])
            return rng.permutation(q).reshape(N, 1)
        q = rng.normal(size=N)
        if zero_mean:
            q = q - q.mean()
        return q.reshape(N, 1)
    if kernel == "stresslet":
        a = rng.normal(size=(N, 3))
        b = rng.normal(size=(N, 3))
        return (a[:, :, None] * b[:, None, :]).reshape(N, 9)
    return rng.normal(size=(N, 3))


def make(name: str, seed: int | None = None, N: int | None = None, kernel: str | None = None) -> Workload:
    """Build one named workload.  ``N`` overrides the point count (same
    distribution and tiling), ``kernel`` picks the kernel of stokes_n2m_rod
    (stresslet by default, or rotlet)."""
    cfgs = {
        # Laplace D=3, unit cube, 2000 uniform points, +-1 charges, 8^3 leaves.
        "laplace_n2k": dict(kernel="laplace", D=3, L=(1.0, 1.0, 1.0), n=(8, 8, 8), N=2000, dist="uniform",
                            sigma=0.05, rc=1.0 / 8, neutral=True, seed=1000),
        # Laplace D=3, unit cube, 1e6 uniform points, 64^3 leaves.
        "laplace_n1m": dict(kernel="laplace", D=3, L=(1.0, 1.0, 1.0), n=(64, 64, 64), N=1_000_000, dist="uniform",
                            seed=1001),
        # Stokeslet D=2, (1,1,4) cuboid, 5e5 points, 70% clustered, 32x32x128 leaves.
        "stokeslet_n500k_clustered": dict(kernel="stokeslet", D=2, L=(1.0, 1.0, 4.0), n=(32, 32, 128), N=500_000,
                                          dist="clustered", seed=1002),
        # Stresslet / rotlet D=1, (32,1,1) cuboid, 2e6 uniform points, 1024x32x32 leaves.
        "stokes_n2m_rod": dict(kernel="stresslet", D=1, L=(32.0, 1.0, 1.0), n=(1024, 32, 32), N=2_000_000,
                               dist="uniform", seed=1003),
    }
    if name not in cfgs:
        raise KeyError(name)
    c = dict(cfgs[name])
    if kernel is not None:
        c["kernel"] = kernel
    if N is not None:
        c["N"] = int(N)
    seed = c.pop("seed") if seed is None else seed
    rng = np.random.default_rng(seed)
    L = c["L"]
    if c["dist"] == "uniform":
        x = _uniform(rng, c["N"], L)
    else:
        x = _clustered(rng, c["N"], L, c["D"])
    rho = _strengths(rng, c["kernel"], c["N"], neutral_charges=c.get("neutral", False))
    h = L[0] / c["n"][0]
    rc = c.get("rc", h)
    sigma = c.get("sigma", h / T_CUT[c["kernel"]])
    return Workload(name=name, kernel=c["kernel"], D=c["D"], L=tuple(L), n=tuple(c["n"]), N=c["N"],
                    sigma=sigma, rc=rc, x=x, rho=rho, seed=seed)


def random_case(seed: int, kernel: str, D: int, L, n, N: int, dist: str = "uniform", rc_frac: float = 1.0,
                sigma_over_rc: float | None = None) -> Workload:
    """Small seeded case for parity tests (any tiling / periodicity)."""
    rng = np.random.default_rng(seed)
    L = tuple(float(v) for v in L)
    x = _uniform(rng, N, L) if dist == "uniform" else _clustered(rng, N, L, D, std=0.05 * min(L))
    rho = _strengths(rng, kernel, N)
    h = min(L[i] / n[i] for i in range(3))
    rc = rc_frac * h
    sigma = rc / T_CUT[kernel] if sigma_over_rc is None else sigma_over_rc * rc
    return Workload(name="rand%d" % seed, kernel=kernel, D=D, L=L, n=tuple(n), N=N, sigma=sigma, rc=rc,
                    x=x, rho=rho, seed=seed)


def cotangent(seed: int, N: int, m_out: int) -> np.ndarray:
    """Seeded cotangent G[N, m_out] for vector-Jacobian products."""
    return np.random.default_rng(seed + 77).normal(size=(N, m_out))
