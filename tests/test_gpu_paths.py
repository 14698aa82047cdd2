"""Bit-exact parity of the stencil kernels' multi-row paths against the
oracle: the 2D kernel with four-row batches per wave (rows >= 4) and the 3D
kernel marching several z-planes per wave, first on small grids with the
launch shape forced through the tuning keys (so that the last band of rows
or planes is partial), then at the sizes where the default launch shape
takes those paths by itself (3D n = 65 and 127, 2D n = 2047)."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2307_00124_amd as P
from tests.test_gpu_ops import STORAGE, star_case

pytestmark = pytest.mark.gpu

KEYS = ("star2d_rows", "star2d_small_n", "star3d_rows", "star3d_small_n")


class tuned:
    """Set tuning keys for the duration of a block, restoring the previous
    values afterwards (also on failure)."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.saved = {k: P.bfp_tuning_get(k) for k in KEYS}
        for k, v in self.kv.items():
            P.bfp_tuning_set(k, v)

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            P.bfp_tuning_set(k, v)
        return False


@pytest.mark.parametrize("ndim,n,rows", [(2, 37, 4), (2, 37, 8), (2, 301, 4), (2, 301, 8),
                                         (3, 19, 2), (3, 19, 4), (3, 37, 4), (3, 37, 32)])
@pytest.mark.parametrize("mode", [P.BFP_SATURATE, P.BFP_NORMALIZE])
@pytest.mark.parametrize("with_y", [False, True])
def test_star_forced_rows(ndim, n, rows, mode, with_y):
    g = np.random.default_rng(ndim * 7919 + n * 31 + rows * 5 + mode * 3 + with_y)
    key = "star2d" if ndim == 2 else "star3d"
    with tuned(**{f"{key}_rows": rows, f"{key}_small_n": 1}):
        for case in range(len(STORAGE)):
            star_case(g, ndim, n, mode, with_y, case, f"{ndim}D n {n} rows {rows}")


@pytest.mark.parametrize("ndim,n", [(3, 65), (3, 127), (2, 2047)])
@pytest.mark.parametrize("mode", [P.BFP_SATURATE, P.BFP_NORMALIZE])
@pytest.mark.parametrize("with_y", [False, True])
def test_star_default_multirow_sizes(ndim, n, mode, with_y):
    """The launch shape the solver uses at these sizes (defaults restored
    first): 3D n >= 64 marches 32 planes per wave, 2D n = 2047 takes eight
    rows per wave in four-row batches. Every storage combination at 3D 65,
    two of them at the larger sizes."""
    g = np.random.default_rng(n * 13 + mode * 3 + with_y)
    with tuned(star2d_rows=0, star2d_small_n=1, star3d_rows=32, star3d_small_n=64):
        cases = range(len(STORAGE)) if n < 100 else (2 * with_y + mode, (2 * with_y + mode + 1) % 4)
        for case in cases:
            star_case(g, ndim, n, mode, with_y, case, f"{ndim}D n {n}")


@pytest.mark.parametrize("ndim,n,rows", [(2, 37, 0), (2, 301, 4), (2, 2047, 0), (3, 19, 0),
                                         (3, 37, 4), (3, 65, 0)])
@pytest.mark.parametrize("mode", [P.BFP_SATURATE, P.BFP_NORMALIZE])
def test_star_y_is_x(ndim, n, rows, mode):
    """The relaxation form c2 A r + c1 r, where y is the block x itself (the
    kernel takes y from the centre values it already holds instead of a
    second stream), for every storage type of r, against the oracle."""
    from oracle import blas
    from oracle.bfp import Scalar
    from tests.gpu_util import assert_block_equal, rand_block, upload
    from tests.test_gpu_ops import fd_A, gamma_pair, quantize_ref
    g = np.random.default_rng(ndim * 31 + n + mode)
    key = "star2d" if ndim == 2 else "star3d"
    kv = {f"{key}_rows": rows, f"{key}_small_n": 1} if rows else {}
    with tuned(**kv):
        for bits in (32, 16, 8):
            w = int(g.integers(2, bits + 1))
            Ad, Ao = fd_A(ndim)
            x = rand_block(g, ndim, n, w, int(g.integers(-30, 30)))
            xd = upload(x, bits)
            c2 = Scalar(-int(g.integers(1, 1 << 15)), int(g.integers(-16, 0)), 16)
            c1 = Scalar(int(g.integers(1, 1 << 15)), int(g.integers(-16, 0)), 16)
            gd, gr = gamma_pair("norm", g, x, xd)
            wz = int(g.integers(2, 33))
            z = P.Vec(ndim, n, wz, 32)
            P.bfp_stencil_apply(Ad, xd, P.scalar(c2.m, c2.e), P.scalar(c1.m, c1.e), xd, wz,
                                mode, gd, z)
            ref = quantize_ref(blas.gemv(Ao, x, x, c2, c1), mode, wz, gr)
            assert_block_equal(z, ref, f"{ndim}D n {n} y = x, storage {bits}")
