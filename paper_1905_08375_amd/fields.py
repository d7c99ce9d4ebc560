"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the nonlocal operator itself: it only draws
fields (horizon, coefficient, state, right-hand sides, displacements) with the
shapes and value distributions of the paper's workloads.  Every draw comes from
``numpy.random.default_rng([190508375, cfg, field])`` so that both sides of a
parity test see bit-identical inputs.

Field recipes (all on the cell-centred grid x_i = (i + 1/2) h, h = 1/n):

* ``grf``: Gaussian random field by spectral synthesis on the periodic n^d grid
  with squared-exponential covariance sigma^2 exp(-r^2 / (2 l^2)); rescaled to
  empirical mean 0 and standard deviation sigma.
* ``voronoi``: piecewise-constant grain field, sites ~ U[0,1]^2, values
  ~ U[lo, hi], nearest site wins (ties to the lowest index).
* ``horizon_*``: the variable horizon delta(x) = m(x) h of each workload.
"""
from __future__ import annotations

import numpy as np

SEED = 190508375


def rng(cfg: int, field: int) -> np.random.Generator:
    return np.random.default_rng([SEED, int(cfg), int(field)])


def nodes(n: int) -> np.ndarray:
    """Cell-centred node coordinates (i + 1/2)/n, i = 0..n-1."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def grf(n: int, dim: int, sigma: float, ell: float, cfg: int, field: int) -> np.ndarray:
    """Gaussian random field (float64, shape (n,)*dim) of std sigma, corr. length ell."""
    g = rng(cfg, field)
    white = g.standard_normal((n,) * dim)
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    kk = np.zeros((n,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = n
        kk = kk + (k1.reshape(shape)) ** 2
    # spectral density of exp(-r^2/(2 l^2)) is proportional to exp(-l^2 |k|^2 / 2)
    amp = np.exp(-0.25 * ell * ell * kk)
    f = np.real(np.fft.ifftn(np.fft.fftn(white) * amp))
    f = f - f.mean()
    sd = f.std()
    return sigma * f / (sd if sd > 0 else 1.0)


def voronoi(n: int, nsites: int, lo: float, hi: float, cfg: int, field: int) -> np.ndarray:
    g = rng(cfg, field)
    sites = g.uniform(0.0, 1.0, size=(nsites, 2))
    vals = g.uniform(lo, hi, size=nsites)
    x = nodes(n)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    best = np.full((n, n), np.inf)
    out = np.zeros((n, n))
    for s in range(nsites):  # strict '<' keeps the lowest index on ties
        d2 = (X1 - sites[s, 0]) ** 2 + (X2 - sites[s, 1]) ** 2
        take = d2 < best
        best = np.where(take, d2, best)
        out = np.where(take, vals[s], out)
    return out


def mesh(n: int, dim: int):
    x = nodes(n)
    return np.meshgrid(*([x] * dim), indexing="ij")


def pad(u: np.ndarray, R: int, value: float = 0.0) -> np.ndarray:
    """Embed u into a collar of width R filled with the volume-constraint value."""
    return np.pad(u, [(R, R)] * u.ndim, mode="constant", constant_values=value)


def padded_coords(n: int, dim: int, R: int):
    x = (np.arange(-R, n + R, dtype=np.float64) + 0.5) / n
    return np.meshgrid(*([x] * dim), indexing="ij")


# ---------------------------------------------------------------- workloads
def diffusion_1d(n: int = 4096, delta: float = 0.01, cfg: int = 1):
    """1D constant horizon, u = sum of 8 sines with N(0,1) amplitudes and 8
    distinct integer frequencies from 1..16 (sin(pi f x) reading)."""
    g = rng(cfg, 0)
    amps = g.standard_normal(8)
    freqs = g.choice(np.arange(1, 17), size=8, replace=False)
    x = nodes(n)
    u = np.zeros(n)
    for a, f in zip(amps, freqs):
        u += a * np.sin(np.pi * f * x)
    delta_f = np.full(n, delta)
    coef = np.ones(n)
    return dict(delta=delta_f, coef=coef, u=u, amps=amps, freqs=freqs)


def horizon_c2(n: int) -> np.ndarray:
    """m(x) = 4 (1 + 0.5 sin 2 pi x1 cos 2 pi x2), delta = m h  (m in [2, 6])."""
    X1, X2 = mesh(n, 2)
    m = 4.0 * (1.0 + 0.5 * np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2))
    return m / n


def diffusion_2d(n: int = 1024, cfg: int = 2):
    delta = horizon_c2(n)
    coef = np.exp(grf(n, 2, 0.5, 0.1, cfg, 1))
    u = grf(n, 2, 1.0, 0.1, cfg, 2)
    return dict(delta=delta, coef=coef, u=u)


def horizon_c3(n: int) -> np.ndarray:
    """m(x) = 7.5 + 4.5 sin 2 pi x1 cos 2 pi x2  (m in [3, 12])."""
    X1, X2 = mesh(n, 2)
    return (7.5 + 4.5 * np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2)) / n


def peridynamic_2d(n: int = 2048, batch: int = 8, R: int = 12, cfg: int = 3):
    """Vector displacement fields u_b = 1e-3 GRF + theta_b J (x - 1/2), b < batch.

    Returns u already padded (the collar carries the same motion), shape
    (batch, 2, n + 2R, n + 2R), plus delta and coef on the n^2 grid."""
    delta = horizon_c3(n)
    coef = voronoi(n, 16, 0.5, 2.0, cfg, 1)
    X1, X2 = padded_coords(n, 2, R)
    g = rng(cfg, 2)
    thetas = g.normal(0.0, 1e-3, size=batch)  # std 1e-3 (variance 1e-6)
    u = np.empty((batch, 2, n + 2 * R, n + 2 * R))
    for b in range(batch):
        r1 = pad(1e-3 * grf(n, 2, 1.0, 0.1, cfg, 10 + 2 * b), R)
        r2 = pad(1e-3 * grf(n, 2, 1.0, 0.1, cfg, 11 + 2 * b), R)
        # J = [[0,-1],[1,0]]: rotation generator about the centre
        u[b, 0] = r1 - thetas[b] * (X2 - 0.5)
        u[b, 1] = r2 + thetas[b] * (X1 - 0.5)
    return dict(delta=delta, coef=coef, u=u, thetas=thetas)


def solve_instance_2d(n: int, inst: int, cfg: int = 4):
    """One batched-solve instance: m(x) = 5 + 3 sin(2 pi (a1 x1 + p1)) cos(2 pi (a2 x2 + p2))."""
    g = rng(cfg, 1000 + inst)
    a = g.integers(1, 3, size=2)
    ph = g.uniform(0.0, 1.0, size=2)
    X1, X2 = mesh(n, 2)
    m = 5.0 + 3.0 * np.sin(2 * np.pi * (a[0] * X1 + ph[0])) * np.cos(2 * np.pi * (a[1] * X2 + ph[1]))
    coef = np.exp(grf(n, 2, 0.5, 0.1, cfg, 2000 + inst))
    b = rng(cfg, 3000 + inst).standard_normal((n, n))
    return dict(delta=m / n, coef=coef, b=b)


def solve_sizes(count: int = 64, cfg: int = 4) -> list:
    g = rng(cfg, 0)
    return [int(v) for v in g.choice([256, 384, 512, 768, 1024], size=count)]


def horizon_c5(n: int) -> np.ndarray:
    """m(x) = 3 + sin 2 pi x1 sin 2 pi x2 sin 2 pi x3  (m in [2, 4])."""
    X1, X2, X3 = mesh(n, 3)
    return (3.0 + np.sin(2 * np.pi * X1) * np.sin(2 * np.pi * X2) * np.sin(2 * np.pi * X3)) / n


def diffusion_3d(n: int = 256, seed_field: int = 0, cfg: int = 5):
    delta = horizon_c5(n)
    coef = np.exp(grf(n, 3, 0.5, 0.1, cfg, 100 + seed_field))
    b = rng(cfg, 200 + seed_field).standard_normal((n, n, n))
    return dict(delta=delta, coef=coef, b=b)


def example1_delta(n: int) -> np.ndarray:
    """The paper's Example 1: constant delta = 1/2 on [0,1]^2."""
    return np.full((n, n), 0.5)


def example2_delta(n: int, delta0: float = 0.25) -> np.ndarray:
    """delta(x) = delta0 (1 + exp(-20 (x - 1/2)^2)) on [0,1] (the paper's 1D heterogeneous horizon)."""
    x = nodes(n)
    return delta0 * (1.0 + np.exp(-20.0 * (x - 0.5) ** 2))
