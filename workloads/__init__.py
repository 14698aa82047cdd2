"""Seeded synthetic inputs for the BFP multigrid workloads.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no arithmetic of the block-floating-point method: it only samples right-hand
sides and manufactured solutions on grids and draws random numbers, so that
both the oracle and the HIP path are fed byte-identical FP64 / integer arrays.

Grids are vertex-centred on the unit square / cube: level j has mesh size
h = 2**-j, n = 2**j - 1 interior points per dimension and a padded array of
(n + 2)**d points whose outer ring holds the homogeneous Dirichlet boundary.
Arrays are C-ordered ``[z][y][x]`` (x fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "padded_side", "coords", "manufactured_f", "manufactured_u",
    "SineModes", "draw_sine_modes", "sine_f", "sine_u",
    "initial_guess", "random_mantissas", "BatchSolve", "batch_trace",
    "Request", "serving_trace", "snap_side",
]


def padded_side(j: int) -> int:
    """Points per dimension of the padded level-j grid (2**j + 1)."""
    return (1 << j) + 1


def coords(j: int) -> np.ndarray:
    """The 2**j + 1 node coordinates k * 2**-j, k = 0..2**j (exact in FP64)."""
    return np.arange(padded_side(j), dtype=np.float64) * (2.0 ** -j)


def _outer(vals: list[np.ndarray]) -> np.ndarray:
    out = vals[0]
    for v in vals[1:]:
        out = np.multiply.outer(v, out)  # later axes are slower: [z][y][x]
    return out


def manufactured_u(j: int, ndim: int) -> np.ndarray:
    """u*(x) = prod_k sin(pi x_k) sampled on the padded level-j grid."""
    s = np.sin(math.pi * coords(j))
    s[0] = 0.0
    s[-1] = 0.0
    return _outer([s] * ndim)


def manufactured_f(j: int, ndim: int) -> np.ndarray:
    """f = d * pi**2 * u*, the right-hand side of -Laplace(u*) = f."""
    return (ndim * math.pi ** 2) * manufactured_u(j, ndim)


@dataclass(frozen=True)
class SineModes:
    """f = sum_i a_i prod_k sin(k_{i,k} pi x_k); k has shape (modes, ndim)."""
    k: np.ndarray
    a: np.ndarray

    @property
    def ndim(self) -> int:
        return int(self.k.shape[1])


def draw_sine_modes(g: np.random.Generator, ndim: int, nmodes: int = 8) -> SineModes:
    """Draw order: kx, ky[, kz] (each ``integers(1, 9, nmodes)``), then
    ``standard_normal(nmodes)`` divided by |k|^2."""
    ks = [g.integers(1, 9, nmodes) for _ in range(ndim)]
    k2 = sum(kk.astype(np.float64) ** 2 for kk in ks)
    a = g.standard_normal(nmodes) / k2
    return SineModes(np.stack(ks, axis=1).astype(np.int64), a)


def sine_f(j: int, modes: SineModes) -> np.ndarray:
    x = coords(j)
    f = np.zeros((padded_side(j),) * modes.ndim)
    for i in range(modes.k.shape[0]):
        parts = []
        for d in range(modes.ndim):
            s = np.sin(math.pi * float(modes.k[i, d]) * x)
            s[0] = 0.0
            s[-1] = 0.0
            parts.append(s)
        f += modes.a[i] * _outer(parts)
    return f


def sine_u(j: int, modes: SineModes) -> np.ndarray:
    """Continuum solution of -Laplace(u) = sine_f: a_i / (pi^2 |k_i|^2) per mode."""
    x = coords(j)
    u = np.zeros((padded_side(j),) * modes.ndim)
    for i in range(modes.k.shape[0]):
        parts = []
        for d in range(modes.ndim):
            s = np.sin(math.pi * float(modes.k[i, d]) * x)
            s[0] = 0.0
            s[-1] = 0.0
            parts.append(s)
        k2 = float(np.sum(modes.k[i].astype(np.float64) ** 2))
        u += (modes.a[i] / (math.pi ** 2 * k2)) * _outer(parts)
    return u


def initial_guess(j: int, ndim: int, seed: int = 0) -> np.ndarray:
    """Uniform[-1, 1] interior values (row-major draw), zero Dirichlet ring."""
    n = (1 << j) - 1
    g = np.random.default_rng(seed)
    out = np.zeros((n + 2,) * ndim)
    out[(slice(1, -1),) * ndim] = g.uniform(-1.0, 1.0, (n,) * ndim)
    return out


def random_mantissas(g: np.random.Generator, shape: tuple[int, ...], w: int,
                     ring: bool = True) -> np.ndarray:
    """Uniform integers in [-2**(w-1), 2**(w-1) - 1] (int64); zero outer ring
    when ``ring`` is set."""
    lo = -(1 << (w - 1))
    hi = (1 << (w - 1)) - 1
    m = g.integers(lo, hi, size=shape, endpoint=True, dtype=np.int64)
    if ring:
        inner = np.zeros(shape, dtype=bool)
        inner[tuple(slice(1, -1) for _ in shape)] = True
        m[~inner] = 0
    return m


@dataclass(frozen=True)
class BatchSolve:
    side: int
    modes: SineModes

    @property
    def level(self) -> int:
        return int(round(math.log2(self.side - 1)))


def batch_trace(count: int = 4096, seed: int = 1,
                sides: tuple[int, ...] = (33, 65, 129, 257)) -> list[BatchSolve]:
    """Independent 2D solves: sides drawn first, then each solve's modes in order."""
    g = np.random.default_rng(seed)
    s = g.choice(np.asarray(sides), count)
    return [BatchSolve(int(si), draw_sine_modes(g, 2)) for si in s]


def snap_side(s: float) -> int:
    """Nearest 2**j + 1 grid side (rounding j = log2(s - 1))."""
    j = int(round(math.log2(s - 1.0)))
    return (1 << j) + 1


@dataclass(frozen=True)
class Request:
    t_arrival: float
    ndim: int
    side: int
    w: int
    modes: SineModes

    @property
    def level(self) -> int:
        return int(round(math.log2(self.side - 1)))


def serving_trace(count: int, rate: float = 2000.0, seed: int = 2) -> list[Request]:
    """Open-loop Poisson arrivals of mixed 2D/3D solves of mixed widths."""
    g = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += g.exponential(1.0 / rate)
        ndim = 2 if g.random() < 0.5 else 3
        if ndim == 2:
            s = math.exp(g.uniform(math.log(65), math.log(1025)))
        else:
            s = math.exp(g.uniform(math.log(33), math.log(129)))
        w = int(g.choice(np.asarray([8, 16, 24, 32])))
        out.append(Request(t, ndim, snap_side(s), w, draw_sine_modes(g, ndim)))
    return out
