"""Finite-difference operators on padded vertex-centred grids, after the
paper's setup S (Appendix C, Algorithm "Setup S to ensure that D = I").

Level j has h = 2^-j, n = 2^j - 1 interior points per dimension and a padded
array of (n + 2)^d points with a zero Dirichlet ring; coarse index I matches
fine index 2I. The unscaled operators are the 5-point (2D) / 7-point (3D)
negative Laplacian A_h = (1/h^2)[2d; -1 ...], bilinear / trilinear nodal
interpolation P, and full weighting 2^-d P^T as the restriction consistent
with finite differences.

Setup S divides every equation by a level scaling s_j so that divisions never
occur in BFP: A' = A_h / s_j, b' = f / s_j and R' = s_c^-1 (2^-d P^T) s_f.
  * 2D: s_j = diag(A_h) = 4/h^2 as in the paper, giving A' = [1; -1/4],
    R' = P^T.
  * 3D: diag(A_h) = 6/h^2 would put -1/6 (not a dyadic rational) into A', so
    the power of two s_j = 8/h^2 is used instead: A' = [3/4; -1/8],
    R' = P^T / 2. The Chebyshev coefficients absorb diag(A') = 3/4 (see
    oracle.mg).
Every scaled operator is an exact dyadic stencil, held here as a BFP matrix
(one exponent, integer taps) at its minimal exact width. Quantizing it to any
wider width (the quant(A), quant(P), quant(R) steps of the V-cycle and FMG)
does not change its value.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .bfp import dyadic_parts, msb


def n_interior(j: int) -> int:
    return (1 << j) - 1


def side(j: int) -> int:
    return (1 << j) + 1


def level_scale(j: int, ndim: int) -> Fraction:
    """s_j: 4/h^2 in 2D (the diagonal of A_h), 8/h^2 in 3D (power of two)."""
    h2 = Fraction(1, 1 << (2 * j))
    return (Fraction(4) if ndim == 2 else Fraction(8)) / h2


def rhs_log2_scale(j: int, ndim: int) -> int:
    """log2(1 / s_j): b' = f * 2^k with k = -2j - 2 (2D) or -2j - 3 (3D)."""
    z, e = dyadic_parts(1 / level_scale(j, ndim))
    assert z == 1
    return e


def _offsets(ndim: int, radius: int = 1):
    return list(itertools.product(range(-radius, radius + 1), repeat=ndim))


def laplacian_taps(j: int, ndim: int) -> dict[tuple, Fraction]:
    """Unscaled (1/h^2)[2d; -1 x 2d] with offsets in array order (z, y, x)."""
    inv_h2 = Fraction(1 << (2 * j))
    taps = {}
    for o in _offsets(ndim):
        l1 = sum(abs(c) for c in o)
        if l1 == 0:
            taps[o] = 2 * ndim * inv_h2
        elif l1 == 1:
            taps[o] = -inv_h2
    return taps


def interpolation_taps(ndim: int) -> dict[tuple, Fraction]:
    """Bilinear / trilinear nodal interpolation weights: a coarse value 1 at
    node 2I gives the fine node 2I + o the weight prod_k (1 or 1/2)."""
    return {o: Fraction(1, 1 << sum(abs(c) for c in o)) for o in _offsets(ndim)}


@dataclass
class Stencil:
    """A constant-coefficient BFP matrix on padded grids: exponent e, integer
    taps (offset -> mantissa, offsets in array order), minimal width w and
    m_A = the maximum number of nonzeros in a row.

    kind 'A': same grid,   out[p] = sum_o t[o] x[p + o]
    kind 'R': fine->coarse, out[I] = sum_o t[o] x[2I + o]
    kind 'P': coarse->fine, out[p] = sum_o t[o] u[p + o], u the coarse block
              placed on the even fine nodes (zeros elsewhere)."""
    kind: str
    ndim: int
    e: int
    taps: dict
    w: int
    m_A: int

    def values(self) -> dict[tuple, Fraction]:
        s = Fraction(2) ** self.e
        return {o: t * s for o, t in self.taps.items()}

    def norm_inf(self) -> Fraction:
        """Largest absolute row sum. For R every interior coarse row holds all
        taps; for A likewise."""
        return sum((abs(v) for v in self.values().values()), Fraction(0))

    def apply(self, xm: np.ndarray) -> np.ndarray:
        """Exact integer row sums over the nonzeros (the espmv rows) for all
        interior output points; the output ring is zero."""
        d = self.ndim
        if xm.ndim != d or len(set(xm.shape)) != 1:
            raise ValueError("expected a padded cubic block")
        nin = xm.shape[0]
        if self.kind == "A":
            nout = nin
            src = xm
            step = 1
        elif self.kind == "R":
            nout = (nin - 1) // 2 + 1
            src = xm
            step = 2
        elif self.kind == "P":
            nout = 2 * (nin - 1) + 1
            src = np.zeros((nout,) * d, dtype=object)
            src[(slice(None, None, 2),) * d] = xm
            step = 1
        else:
            raise ValueError(self.kind)
        out = np.zeros((nout,) * d, dtype=object)
        ni = nout - 2
        if ni <= 0:
            return out
        acc = np.zeros((ni,) * d, dtype=object)
        for o, t in self.taps.items():
            if t == 0:
                continue
            sl = tuple(slice(step * 1 + c, step * 1 + c + step * (ni - 1) + 1, step)
                       for c in o)
            acc = acc + t * src[sl]
        out[(slice(1, -1),) * d] = acc
        return out


def to_stencil(kind: str, ndim: int, taps: dict[tuple, Fraction], m_A: int) -> Stencil:
    """Minimal exact BFP representation of dyadic taps: the largest exponent
    e with every tap an integer multiple of 2^e, width = max msb."""
    parts = {o: dyadic_parts(v) for o, v in taps.items() if v != 0}
    e = min(pe for _, pe in parts.values())
    ints = {o: z << (pe - e) for o, (z, pe) in parts.items()}
    while all(v % 2 == 0 for v in ints.values()):
        ints = {o: v // 2 for o, v in ints.items()}
        e += 1
    w = max(msb(v) for v in ints.values())
    return Stencil(kind, ndim, e, ints, w, m_A)


def scaled_A(j: int, ndim: int) -> Stencil:
    """A' = A_h / s_j."""
    s = level_scale(j, ndim)
    taps = {o: v / s for o, v in laplacian_taps(j, ndim).items()}
    return to_stencil("A", ndim, taps, 2 * ndim + 1)


def prolongation(ndim: int) -> Stencil:
    return to_stencil("P", ndim, interpolation_taps(ndim), 1 << ndim)


def scaled_R(j_fine: int, ndim: int) -> Stencil:
    """R' = s_c^-1 (2^-d P^T) s_f from fine level j to level j - 1. P^T has
    the same taps as P (the interpolation weights are symmetric)."""
    sf = level_scale(j_fine, ndim)
    sc = level_scale(j_fine - 1, ndim)
    scale = sf / sc / (1 << ndim)
    taps = {o: v * scale for o, v in interpolation_taps(ndim).items()}
    return to_stencil("R", ndim, taps, 3 ** ndim)
