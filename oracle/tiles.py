"""Sub-maximal block sizes (Section 2, Remark "Block size").

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU baseline; the product never imports, links or runs anything here.

The paper keeps one exponent per vector (the maximal block) and remarks that
smaller blocks are the worst case's relaxation: a block of size 1 is
floating point, and the results extend to any size in between. Here a grid
vector's interior points are split along the fastest axis of every grid row
into blocks ("tiles") of T consecutive points; the last tile of a row holds
n mod T points when T does not divide n. Every tile is a BFP tuple of its
own (exponent, w-bit mantissas); the zero Dirichlet ring belongs to no tile
and is zero.

Every operation forms the exact rational result of each interior point by
its plain definition and quantizes each output tile on its own with the
normalized floor quantization Q_w of Section 2 (the result Algorithm 1
returns, applied per tile): e = max_i nu(z_i) - w over the tile's nonzero
values, m_i = floor(z_i / 2^e).

Readings (listed in the design notes):
  * an all-zero tile has exponent 1 - w (the exponent Q_w gives a zero
    block; with one block per vector the exponent of a zero qcomp result
    depends on e_z*, which a tile of mixed operand exponents does not have);
  * exact range: an operation computes a point exactly when the exponents of
    the operand tiles it draws from (each plus its coefficient's exponent)
    lie within SPREAD = 60 of each other; a point beyond that is counted and
    set to zero. Ring neighbours carry no exponent (their value is zero).
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .bfp import Scalar, floor_div_pow2, nu

SPREAD = 60


def tile_count(n: int, T: int) -> int:
    return -(-n // T)


@dataclass
class Tiled:
    """A tiled BFP grid vector: m is the padded (n+2)^ndim object array of
    mantissas (ring zero), e the exponent of every tile, shape
    (n^(ndim-1), ceil(n/T)): row r = (z-1) n + (y-1) (3D) or y - 1 (2D),
    tile t holds x = t T + 1 .. min((t+1) T, n)."""
    ndim: int
    n: int
    T: int
    w: int
    e: np.ndarray
    m: np.ndarray

    def tile_exp(self, p: tuple) -> int:
        """Exponent of the tile holding interior point p (padded indices)."""
        r, t = tile_index(self.ndim, self.n, self.T, p)
        return int(self.e[r, t])

    def values(self) -> np.ndarray:
        out = np.zeros(self.m.shape, dtype=object)
        for p in interior(self.ndim, self.n):
            out[p] = Fraction(int(self.m[p])) * Fraction(2) ** self.tile_exp(p)
        return out

    def to_f64(self) -> np.ndarray:
        return np.vectorize(float, otypes=[np.float64])(self.values())


def interior(ndim: int, n: int):
    """Interior points in row-major order (padded indices)."""
    rng = range(1, n + 1)
    if ndim == 2:
        for y in rng:
            for x in rng:
                yield (y, x)
    else:
        for z in rng:
            for y in rng:
                for x in rng:
                    yield (z, y, x)


def tile_index(ndim: int, n: int, T: int, p: tuple) -> tuple[int, int]:
    row = (p[0] - 1) * n + (p[1] - 1) if ndim == 3 else p[0] - 1
    return row, (p[-1] - 1) // T


def quantize(values: np.ndarray, ndim: int, n: int, T: int, w: int) -> Tiled:
    """Q_w of every tile of a padded grid of exact dyadic values (the ring
    is ignored and comes out zero)."""
    if T < 1 or w < 1:
        raise ValueError("need T >= 1 and w >= 1")
    rows = n ** (ndim - 1)
    groups: dict[tuple, list] = {}
    for p in interior(ndim, n):
        groups.setdefault(tile_index(ndim, n, T, p), []).append(p)
    e = np.zeros((rows, tile_count(n, T)), dtype=np.int64)
    m = np.zeros(values.shape, dtype=object)
    for (r, t), pts in groups.items():
        nz = [Fraction(values[p]) for p in pts if Fraction(values[p]) != 0]
        et = (max(nu(v) for v in nz) - w) if nz else 1 - w
        e[r, t] = et
        for p in pts:
            m[p] = floor_div_pow2(Fraction(values[p]), et)
    return Tiled(ndim, n, T, w, e, m)


def from_f64(x: np.ndarray, T: int, w: int) -> Tiled:
    """Tile-wise quant of a padded FP64 grid (FP64 values are exact
    dyadics); the ring of x is not read."""
    x = np.asarray(x, dtype=np.float64)
    ndim, n = x.ndim, x.shape[0] - 2
    if not np.all(np.isfinite(x[(slice(1, -1),) * ndim])):
        raise ValueError("non-finite FP64 input")
    vals = np.zeros(x.shape, dtype=object)
    for p in interior(ndim, n):
        vals[p] = Fraction(float(x[p]))
    return quantize(vals, ndim, n, T, w)


def _combine(terms: list[tuple[int, int]]):
    """Exact sum of terms (integer, exponent) as a Fraction, or None when the
    exponents spread beyond SPREAD."""
    if not terms:
        return Fraction(0)
    exps = [e for _, e in terms]
    if max(exps) - min(exps) > SPREAD:
        return None
    return sum((Fraction(v) * Fraction(2) ** e for v, e in terms), Fraction(0))


def star_point(A, n: int, p: tuple, xm, xe, alpha: Scalar, beta: Scalar | None = None,
               ym=None, ye=None):
    """Exact value of alpha A x (+ beta y) at interior point p, or None when
    its terms spread beyond the exact range. xm(q), xe(q) give x's mantissa
    and tile exponent at interior point q (ym, ye likewise for y)."""
    terms = []
    for o, t in A.taps.items():
        if t == 0:
            continue
        q = tuple(pi + oi for pi, oi in zip(p, o))
        if any(c < 1 or c > n for c in q):
            continue   # ring: zero, no exponent
        terms.append((alpha.m * t * int(xm(q)), alpha.e + A.e + int(xe(q))))
    if ym is not None:
        terms.append((beta.m * int(ym(p)), beta.e + int(ye(p))))
    return _combine(terms)


def stencil_apply(A, x: Tiled, alpha: Scalar, beta: Scalar | None, y: Tiled | None,
                  w_out: int) -> tuple[Tiled, int]:
    """z = alpha A x (+ beta y) on the interior, every output tile Q_w_out of
    its exact values; A is a star stencil of kind 'A' (the oracle.fd
    Stencil). Returns the result (tiled like x) and the number of points
    beyond the exact range."""
    if A.kind != "A" or any(sum(abs(c) for c in o) > 1 for o, t in A.taps.items() if t):
        raise ValueError("tiled stencils: star stencils of kind A only")
    if y is not None and (y.n != x.n or y.T != x.T or y.ndim != x.ndim):
        raise ValueError("y must be tiled like x")
    d, n = x.ndim, x.n
    exact = np.zeros(x.m.shape, dtype=object)
    bad = 0
    for p in interior(d, n):
        v = star_point(A, n, p, lambda q: x.m[q], x.tile_exp, alpha, beta,
                       (lambda q: y.m[q]) if y is not None else None,
                       y.tile_exp if y is not None else None)
        if v is None:
            bad += 1
            v = Fraction(0)
        exact[p] = v
    return quantize(exact, d, n, x.T, w_out), bad


def axpby(alpha: Scalar, x: Tiled, beta: Scalar, y: Tiled, w_out: int) -> tuple[Tiled, int]:
    """z = alpha x + beta y point by point, every output tile Q_w_out of its
    exact values. Returns the result and the points beyond the exact range."""
    if y.n != x.n or y.T != x.T or y.ndim != x.ndim:
        raise ValueError("x and y must be tiled alike")
    exact = np.zeros(x.m.shape, dtype=object)
    bad = 0
    for p in interior(x.ndim, x.n):
        v = _combine([(alpha.m * int(x.m[p]), alpha.e + x.tile_exp(p)),
                      (beta.m * int(y.m[p]), beta.e + y.tile_exp(p))])
        if v is None:
            bad += 1
            v = Fraction(0)
        exact[p] = v
    return quantize(exact, x.ndim, x.n, x.T, w_out), bad
