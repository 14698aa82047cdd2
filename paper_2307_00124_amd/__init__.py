"""BFP multigrid on MI355X: Python binding of libbfpmg.so.

Thin marshalling over the C-ABI declared in include/bfpmg.h: PyTorch supplies
device memory and the stream, every computation runs in the library's HIP
kernels. Function names match the C entry points.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import abi
from .abi import (BFP_GAMMA_EXPLICIT, BFP_GAMMA_NORM, BFP_GAMMA_SUM, BFP_META_EXP,
                  BFP_META_FLAGS, BFP_META_MAX, BFP_META_MIN, BFP_META_MU, BFP_META_SAT,
                  BFP_META_SLOTS, BFP_NORMALIZE, BFP_SATURATE, BFP_STENCIL_A, BFP_STENCIL_P,
                  BFP_STENCIL_R, MG_MAX_LEVELS, MG_POLICY_NN, MG_POLICY_NN_IR_FIRST2_Q,
                  MG_POLICY_NN_IR_FIRST_Q, MG_POLICY_NN_IR_Q, MG_POLICY_Q, BFPError, check,
                  lib)

__all__ = [
    "Vec", "Stencil", "scalar", "gamma_norm", "gamma_sum", "gamma_explicit", "Hierarchy",
    "bfp_layout", "bfp_vec_init", "bfp_vec_assign", "bfp_meta_reset", "mg_params_init", "bfp_vec_from_f64", "bfp_vec_to_f64",
    "bfp_vec_check", "bfp_stencil_apply", "bfp_residual", "bfp_axpy", "bfp_sub", "bfp_dot",
    "bfp_normalize", "bfp_saturate_truncate", "bfp_cheby_coeffs", "BFPError",
    "BFP_NORMALIZE", "BFP_SATURATE", "BFP_STENCIL_A", "BFP_STENCIL_R", "BFP_STENCIL_P",
    "MG_POLICY_Q", "MG_POLICY_NN", "MG_POLICY_NN_IR_FIRST_Q", "MG_POLICY_NN_IR_FIRST2_Q",
    "MG_POLICY_NN_IR_Q", "lib", "Tiles", "bfp_tiles_from_f64", "bfp_tiles_to_f64",
    "bfp_tiles_stencil_apply", "bfp_tiles_axpby",
]

_DTYPES = {8: torch.int8, 16: torch.int16, 32: torch.int32}


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def storage_for(w: int) -> int:
    return 8 if w <= 8 else 16 if w <= 16 else 32


def bfp_layout(ndim: int, n: int, storage_bits: int) -> tuple[int, int]:
    pitch = C.c_int64()
    nbytes = C.c_size_t()
    check(lib.bfp_layout(ndim, n, storage_bits, C.byref(pitch), C.byref(nbytes)), "bfp_layout")
    return pitch.value, nbytes.value


class Vec:
    """A BFP block (one exponent, w-bit mantissas) on a padded grid in device
    memory: a byte buffer of row-pitched mantissas and 16 int64 of metadata."""

    def __init__(self, ndim: int, n: int, w: int, storage_bits: int | None = None,
                 device: str | torch.device = "cuda", init: bool = True, _view=None):
        if _view is not None:
            self.c, self._owner = _view
            self.buf = None
            self.meta = None
            return
        bits = storage_bits or storage_for(w)
        pitch, nbytes = bfp_layout(ndim, n, bits)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.meta = torch.empty(BFP_META_SLOTS, dtype=torch.int64, device=device)
        self.c = abi.bfp_vec(self.buf.data_ptr(), self.meta.data_ptr(), w, bits, ndim, n, pitch)
        self._owner = None
        if init:
            bfp_vec_init(self)

    @classmethod
    def view(cls, c_vec: abi.bfp_vec, owner) -> "Vec":
        return cls(0, 0, 0, _view=(c_vec, owner))

    @property
    def ndim(self) -> int:
        return self.c.ndim

    @property
    def n(self) -> int:
        return self.c.n

    @property
    def w(self) -> int:
        return self.c.w

    @property
    def storage_bits(self) -> int:
        return self.c.storage_bits

    def _raw(self) -> torch.Tensor:
        """The mantissa buffer as a typed device tensor (rows x pitch)."""
        rows = (self.n + 2) ** (self.ndim - 1)
        nbytes = rows * self.c.pitch * self.storage_bits // 8
        if self.buf is not None:
            b = self.buf
        else:
            b = _wrap_device_bytes(self.c.mant, nbytes, self._owner)
        return b[:nbytes].view(_DTYPES[self.storage_bits]).view(rows, self.c.pitch)

    def mantissas(self) -> torch.Tensor:
        """Device view of the (n+2)^ndim mantissas (ring included)."""
        side = self.n + 2
        return self._raw()[:, :side].reshape((side,) * self.ndim)

    def padding(self) -> torch.Tensor:
        return self._raw()[:, self.n + 2:]

    def meta_tensor(self) -> torch.Tensor:
        if self.meta is not None:
            return self.meta
        return _wrap_device_bytes(self.c.meta, BFP_META_SLOTS * 8, self._owner).view(torch.int64)

    def host_meta(self) -> list[int]:
        return [int(v) for v in self.meta_tensor().cpu().tolist()]

    @property
    def exp(self) -> int:
        return self.host_meta()[BFP_META_EXP]


def _wrap_device_bytes(ptr: int, nbytes: int, owner) -> torch.Tensor:
    """A uint8 tensor aliasing device memory inside a torch-owned arena."""
    arena: torch.Tensor = owner.arena
    base = arena.data_ptr()
    off = int(ptr) - base
    if off < 0 or off + nbytes > arena.numel():
        raise ValueError("pointer outside the owning arena")
    return arena[off:off + nbytes]


@dataclass
class Stencil:
    """Constant-coefficient BFP matrix: exponent and 3^ndim integer taps
    (index ((oz+1)*3 + (oy+1))*3 + (ox+1), 2D: (oy+1)*3 + (ox+1))."""
    ndim: int
    kind: int
    exp: int
    taps: list
    w: int = 0

    def c(self) -> abi.bfp_stencil:
        s = abi.bfp_stencil()
        s.ndim, s.kind, s.exp = self.ndim, self.kind, self.exp
        width = self.w or max((abs(t) * 2).bit_length() for t in self.taps)
        s.w = width
        for i, t in enumerate(self.taps):
            s.taps[i] = int(t)
        return s


def scalar(m: int, e: int, w: int | None = None) -> abi.bfp_scalar:
    if w is None:
        w = ((m if m >= 0 else ~m).bit_length()) + 1
    return abi.bfp_scalar(m, e, w)


def gamma_norm(a: Vec, c: abi.bfp_scalar | None = None) -> abi.bfp_gamma:
    g = abi.bfp_gamma()
    g.rule = BFP_GAMMA_NORM
    g.a_meta = a.c.meta
    g.c = c if c is not None else scalar(1, 0)
    return g


def gamma_sum(a: Vec, b: Vec) -> abi.bfp_gamma:
    g = abi.bfp_gamma()
    g.rule = BFP_GAMMA_SUM
    g.a_meta = a.c.meta
    g.b_meta = b.c.meta
    return g


def gamma_explicit(m: int, e: int) -> abi.bfp_gamma:
    g = abi.bfp_gamma()
    g.rule = BFP_GAMMA_EXPLICIT
    g.c = scalar(m, e)
    return g


def _opt(x):
    return C.byref(x) if x is not None else None


def _vc(v: Vec | None):
    return C.byref(v.c) if v is not None else None


# ------------------------------------------------------------ C entry points --

def bfp_vec_init(v: Vec, stream=None) -> None:
    check(lib.bfp_vec_init(C.byref(v.c), _stream(stream)), "bfp_vec_init")


def bfp_vec_assign(v: Vec, exp: int, stream=None) -> None:
    check(lib.bfp_vec_assign(C.byref(v.c), int(exp), _stream(stream)), "bfp_vec_assign")


def bfp_meta_reset(meta: torch.Tensor, stream=None) -> None:
    check(lib.bfp_meta_reset(_ptr(meta), _stream(stream)), "bfp_meta_reset")


def bfp_vec_from_f64(src: torch.Tensor, log2_scale: int, dst: Vec, stream=None) -> None:
    if src.dtype != torch.float64 or not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous float64 device tensor")
    if src.numel() != (dst.n + 2) ** dst.ndim:
        raise ValueError("src must hold (n+2)^ndim values")
    check(lib.bfp_vec_from_f64(_ptr(src), int(log2_scale), C.byref(dst.c), _stream(stream)),
          "bfp_vec_from_f64")


def bfp_vec_to_f64(src: Vec, dst: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if dst is None:
        dst = torch.empty((src.n + 2,) * src.ndim, dtype=torch.float64, device="cuda")
    if dst.dtype != torch.float64 or not dst.is_contiguous() or dst.numel() != (src.n + 2) ** src.ndim:
        raise ValueError("dst must be a contiguous float64 tensor of (n+2)^ndim")
    check(lib.bfp_vec_to_f64(C.byref(src.c), _ptr(dst), _stream(stream)), "bfp_vec_to_f64")
    return dst


def bfp_vec_check(v: Vec, stream=None) -> None:
    check(lib.bfp_vec_check(C.byref(v.c), _stream(stream)), "bfp_vec_check")


def bfp_stencil_apply(A: Stencil, x: Vec, alpha, beta, y: Vec | None, w_out: int, mode: int,
                      gamma, z: Vec, stream=None) -> None:
    Ac = A.c()
    check(lib.bfp_stencil_apply(C.byref(Ac), C.byref(x.c), _opt(alpha), _opt(beta), _vc(y),
                                w_out, mode, _opt(gamma), C.byref(z.c), _stream(stream)),
          "bfp_stencil_apply")


def bfp_residual(A: Stencil, x: Vec, b: Vec, w_out: int, mode: int, gamma, r: Vec,
                 stream=None) -> None:
    Ac = A.c()
    check(lib.bfp_residual(C.byref(Ac), C.byref(x.c), C.byref(b.c), w_out, mode, _opt(gamma),
                           C.byref(r.c), _stream(stream)), "bfp_residual")


def bfp_axpy(alpha, x: Vec, beta, y: Vec, w_out: int, mode: int, gamma, z: Vec,
             stream=None) -> None:
    check(lib.bfp_axpy(C.byref(alpha), C.byref(x.c), C.byref(beta), C.byref(y.c), w_out, mode,
                       _opt(gamma), C.byref(z.c), _stream(stream)), "bfp_axpy")


def bfp_sub(x: Vec, y: Vec, w_out: int, mode: int, gamma, z: Vec, stream=None) -> None:
    check(lib.bfp_sub(C.byref(x.c), C.byref(y.c), w_out, mode, _opt(gamma), C.byref(z.c),
                      _stream(stream)), "bfp_sub")


def bfp_dot(x: Vec, y: Vec, out: torch.Tensor, stream=None) -> None:
    if out.dtype != torch.int64 or out.numel() < BFP_META_SLOTS:
        raise ValueError(f"out must be an int64 device tensor of {BFP_META_SLOTS} zeroed slots")
    check(lib.bfp_dot(C.byref(x.c), C.byref(y.c), _ptr(out), _stream(stream)), "bfp_dot")


def bfp_stream_copy(src: torch.Tensor, dst: torch.Tensor, nontemporal: bool = False,
                    stream=None) -> None:
    """bfp_stream_copy: dst <- src (whole tensors of equal byte size), the
    library's plain streaming copy (the bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("src and dst must be device tensors of the same size in bytes")
    check(lib.bfp_stream_copy(_ptr(src), _ptr(dst), nbytes, int(nontemporal), _stream(stream)),
          "bfp_stream_copy")


def bfp_normalize(x: Vec, w_out: int, out: Vec, stream=None) -> None:
    check(lib.bfp_normalize(C.byref(x.c), w_out, C.byref(out.c), _stream(stream)),
          "bfp_normalize")


def bfp_saturate_truncate(x: Vec, w_out: int, gamma, out: Vec, stream=None) -> None:
    check(lib.bfp_saturate_truncate(C.byref(x.c), w_out, _opt(gamma), C.byref(out.c),
                                    _stream(stream)), "bfp_saturate_truncate")


# ------------------------------------------------ sub-maximal block sizes --

class Tiles:
    """A tiled BFP grid vector (bfp_tiles): padded row-pitched mantissas and
    one int32 exponent per tile of T consecutive row points."""

    def __init__(self, ndim: int, n: int, T: int, w: int, storage_bits: int | None = None,
                 device: str | torch.device = "cuda", init: bool = True):
        bits = storage_bits or storage_for(w)
        pitch, mbytes, ebytes = C.c_int64(), C.c_size_t(), C.c_size_t()
        check(lib.bfp_tiles_layout(ndim, n, T, bits, C.byref(pitch), C.byref(mbytes),
                                   C.byref(ebytes)), "bfp_tiles_layout")
        self.buf = torch.empty(mbytes.value, dtype=torch.uint8, device=device)
        self.exps = torch.empty(ebytes.value // 4, dtype=torch.int32, device=device)
        self.c = abi.bfp_tiles(self.buf.data_ptr(), self.exps.data_ptr(), w, bits, ndim, n, T,
                               pitch.value)
        if init:
            check(lib.bfp_tiles_init(C.byref(self.c), _stream(None)), "bfp_tiles_init")

    ndim = property(lambda self: self.c.ndim)
    n = property(lambda self: self.c.n)
    T = property(lambda self: self.c.T)
    w = property(lambda self: self.c.w)
    storage_bits = property(lambda self: self.c.storage_bits)

    def mantissas(self) -> torch.Tensor:
        """Device view of the (n+2)^ndim mantissas (ring included)."""
        rows = (self.n + 2) ** (self.ndim - 1)
        side = self.n + 2
        raw = self.buf[:rows * self.c.pitch * self.storage_bits // 8]
        return raw.view(_DTYPES[self.storage_bits]).view(rows, self.c.pitch)[:, :side].reshape(
            (side,) * self.ndim)

    def exponents(self) -> torch.Tensor:
        """Device view of the tile exponents, (n^(ndim-1), ceil(n/T))."""
        return self.exps.view(self.n ** (self.ndim - 1), -(-self.n // self.T))


def bfp_tiles_from_f64(src: torch.Tensor, dst: Tiles, status: torch.Tensor | None = None,
                       stream=None) -> None:
    if src.dtype != torch.float64 or not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous float64 device tensor")
    if src.numel() != (dst.n + 2) ** dst.ndim:
        raise ValueError("src must hold (n+2)^ndim values")
    check(lib.bfp_tiles_from_f64(_ptr(src), C.byref(dst.c), _opt_ptr(status), _stream(stream)),
          "bfp_tiles_from_f64")


def bfp_tiles_to_f64(src: Tiles, dst: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if dst is None:
        dst = torch.zeros((src.n + 2,) * src.ndim, dtype=torch.float64, device="cuda")
    if dst.dtype != torch.float64 or not dst.is_contiguous() or dst.numel() != (src.n + 2) ** src.ndim:
        raise ValueError("dst must be a contiguous float64 tensor of (n+2)^ndim")
    check(lib.bfp_tiles_to_f64(C.byref(src.c), _ptr(dst), _stream(stream)), "bfp_tiles_to_f64")
    return dst


def bfp_tiles_stencil_apply(A: Stencil, x: Tiles, alpha, beta, y: Tiles | None, z: Tiles,
                            status: torch.Tensor | None = None, stream=None) -> None:
    Ac = A.c()
    check(lib.bfp_tiles_stencil_apply(C.byref(Ac), C.byref(x.c), _opt(alpha), _opt(beta),
                                      C.byref(y.c) if y is not None else None, C.byref(z.c),
                                      _opt_ptr(status), _stream(stream)),
          "bfp_tiles_stencil_apply")


def bfp_tiles_axpby(alpha, x: Tiles, beta, y: Tiles, z: Tiles, status: torch.Tensor | None = None,
                    stream=None) -> None:
    check(lib.bfp_tiles_axpby(_opt(alpha), C.byref(x.c), _opt(beta), C.byref(y.c), C.byref(z.c),
                              _opt_ptr(status), _stream(stream)), "bfp_tiles_axpby")


def _opt_ptr(t: torch.Tensor | None):
    return _ptr(t) if t is not None else None


# ------------------------------------ finite-element model problems --

class FEHierarchy:
    """fe_hierarchy: the 1D B-spline FE model problems of Section 6 in BFP
    FMG. K, P: per level, banded matrices of Fractions (objects with nrows,
    ncols, col0, vals as workloads.fe.Band; P[0] unused); F: per level, the
    FP64 load vectors (host arrays); widths: dicts level -> width."""

    def __init__(self, m: int, L: int, N: int, K: list, P: list, F: list, w_check: dict,
                 w_work: dict, w_inner: dict, eta=(23, 100), stream=None):
        import numpy as np
        prm = abi.fe_params()
        prm.m, prm.L, prm.N = m, L, N
        prm.eta_num, prm.eta_den = eta
        for j in range(1, L + 1):
            prm.w_check[j], prm.w_work[j], prm.w_inner[j] = w_check[j], w_work[j], w_inner[j]
        self._keep = []

        def band(B):
            width = max(len(r) for r in B.vals)
            width = min(width, B.ncols)
            col0 = np.zeros(B.nrows, dtype=np.int32)
            num = np.zeros((B.nrows, width), dtype=np.int64)
            den = np.ones((B.nrows, width), dtype=np.int64)
            for i, row in enumerate(B.vals):
                c = max(0, min(B.col0[i], B.ncols - width))
                col0[i] = c
                for t, v in enumerate(row):
                    at = B.col0[i] + t - c
                    if v != 0:
                        num[i, at], den[i, at] = v.numerator, v.denominator
            self._keep += [col0, num, den]
            return abi.fe_rational_band(B.nrows, B.ncols, width, col0.ctypes.data,
                                        num.ctypes.data, den.ctypes.data)
        Ks = (abi.fe_rational_band * L)(*[band(K[j]) for j in range(L)])
        Ps = (abi.fe_rational_band * L)(*([abi.fe_rational_band()] +
                                           [band(P[j]) for j in range(1, L)]))
        Fs = [np.ascontiguousarray(f, dtype=np.float64) for f in F]
        self._keep += Fs
        Fp = (C.c_void_p * L)(*[f.ctypes.data for f in Fs])
        h = C.c_void_p()
        check(lib.fe_hierarchy_create(C.byref(prm), Ks, Ps, Fp, _stream(stream), C.byref(h)),
              "fe_hierarchy_create")
        self.h = h
        self.L = L

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.fe_hierarchy_destroy(self.h)
            self.h = None

    def fmg(self, stream=None) -> None:
        check(lib.fe_fmg(self.h, _stream(stream)), "fe_fmg")

    def get(self, level: int, which: int = 0):
        """(mantissas with the two zero ends, exponent) of a block."""
        import numpy as np
        e, n = C.c_int64(), C.c_int()
        check(lib.fe_get(self.h, level, which, None, C.byref(e), C.byref(n)), "fe_get")
        out = np.zeros(n.value + 2, dtype=np.int32)
        check(lib.fe_get(self.h, level, which, out.ctypes.data, C.byref(e), C.byref(n)), "fe_get")
        return out, e.value

    def coefficients(self):
        c1, c2 = abi.bfp_scalar(), abi.bfp_scalar()
        check(lib.fe_coefficients(self.h, C.byref(c1), C.byref(c2)), "fe_coefficients")
        return (c1.m, c1.exp), (c2.m, c2.exp)

    def counters(self):
        b, n = C.c_double(), C.c_int64()
        check(lib.fe_counters(self.h, C.byref(b), C.byref(n)), "fe_counters")
        return b.value, n.value


def bfp_tuning_set(key: str, value: int) -> None:
    check(lib.bfp_tuning_set(key.encode(), int(value)), "bfp_tuning_set")


def bfp_tuning_get(key: str) -> int:
    v = C.c_int(0)
    check(lib.bfp_tuning_get(key.encode(), C.byref(v)), "bfp_tuning_get")
    return int(v.value)


def bfp_cheby_coeffs(rho: tuple[int, int], eta: tuple[int, int], scale: tuple[int, int] = (1, 1),
                     w: int = 16) -> tuple[abi.bfp_scalar, abi.bfp_scalar]:
    c1, c2 = abi.bfp_scalar(), abi.bfp_scalar()
    check(lib.bfp_cheby_coeffs(rho[0], rho[1], eta[0], eta[1], scale[0], scale[1], w,
                               C.byref(c1), C.byref(c2)), "bfp_cheby_coeffs")
    return c1, c2


# ------------------------------------------------------------ multigrid ---

class Hierarchy:
    """A solver hierarchy in a torch-allocated device arena (mg_* calls)."""

    def __init__(self, params: abi.mg_params, device="cuda", stream=None):
        self.params = params
        nbytes = lib.mg_hierarchy_bytes(C.byref(params))
        if nbytes == 0:
            raise BFPError(abi.BFP_EINVAL, "mg_hierarchy_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self.arena = self.arena[off:off + nbytes]
        h = C.c_void_p()
        check(lib.mg_hierarchy_create(C.byref(params), _ptr(self.arena), nbytes, _stream(stream),
                                      C.byref(h)), "mg_hierarchy_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and lib is not None:   # not at interpreter exit
            lib.mg_hierarchy_destroy(h)
            self.h = None

    def _check_f64(self, level: int, f: torch.Tensor, what: str) -> None:
        side = (1 << level) + 1
        if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous():
            raise ValueError(f"{what} must be a contiguous float64 device tensor")
        if f.numel() != side ** self.params.ndim:
            raise ValueError(f"{what} must hold the padded level-{level} grid "
                             f"({side}^{self.params.ndim} values), not {f.numel()}")

    def set_rhs(self, level: int, f: torch.Tensor, stream=None) -> None:
        if 1 <= level <= self.params.L:
            self._check_f64(level, f, "f")
        check(lib.mg_set_rhs(self.h, level, _ptr(f), _stream(stream)), "mg_set_rhs")

    def fmg_f64(self, rhs: list, stream=None) -> None:
        """mg_fmg_f64: quantize the right-hand sides rhs[j-1] of levels
        j = 1..L (FP64, padded grids) and run FMG, in one call."""
        L = self.params.L
        if len(rhs) != L:
            raise ValueError(f"need {L} right-hand sides, got {len(rhs)}")
        for j, f in enumerate(rhs, start=1):
            self._check_f64(j, f, f"rhs[{j - 1}]")
        ptrs = (C.c_void_p * L)(*[f.data_ptr() for f in rhs])
        check(lib.mg_fmg_f64(self.h, ptrs, _stream(stream)), "mg_fmg_f64")

    def set_x(self, level: int, x0: torch.Tensor, stream=None) -> None:
        if 1 <= level <= self.params.L:
            self._check_f64(level, x0, "x0")
        check(lib.mg_set_x(self.h, level, _ptr(x0), _stream(stream)), "mg_set_x")

    def fmg(self, stream=None) -> None:
        check(lib.mg_fmg(self.h, _stream(stream)), "mg_fmg")

    def ir_safe(self, level: int, iters: int, q_iters: int = 2, theta=(1, 0),
                stream=None) -> int:
        """mg_ir_safe: IR-V with the qcomp fallback; theta = (num, k) stands
        for num / 2^k. Returns the number of iterations that ran the
        fallback."""
        sw = C.c_int(0)
        check(lib.mg_ir_safe(self.h, level, iters, q_iters, int(theta[0]), int(theta[1]),
                             C.byref(sw), _stream(stream)), "mg_ir_safe")
        return sw.value

    def diagnostics(self, reset: bool = False, stream=None):
        """mg_diag_read: the solve diagnostics as an int64 numpy array
        [level 0..MG_MAX_LEVELS][site][bin] (synchronizes `stream`)."""
        import numpy as np
        out = np.zeros((abi.MG_MAX_LEVELS + 1, abi.MG_DIAG_SITES, abi.MG_DIAG_BINS), dtype=np.int64)
        check(lib.mg_diag_read(self.h, out.ctypes.data_as(C.c_void_p), int(reset), _stream(stream)),
              "mg_diag_read")
        return out

    def ir(self, level: int, iters: int, stream=None) -> None:
        check(lib.mg_ir(self.h, level, iters, _stream(stream)), "mg_ir")

    def vcycle(self, level: int, r: Vec, stream=None) -> Vec:
        y = abi.bfp_vec()
        check(lib.mg_vcycle(self.h, level, C.byref(r.c), C.byref(y), _stream(stream)),
              "mg_vcycle")
        return Vec.view(y, self)

    def get_vec(self, level: int, which: int = 0) -> Vec:
        v = abi.bfp_vec()
        check(lib.mg_get_vec(self.h, level, which, C.byref(v)), "mg_get_vec")
        return Vec.view(v, self)

    def counters(self) -> tuple[float, int]:
        b = C.c_double()
        n = C.c_int64()
        check(lib.mg_counters(self.h, C.byref(b), C.byref(n)), "mg_counters")
        return b.value, n.value

    def autotune(self, reps: int = 20, stream=None) -> dict:
        """mg_autotune: per-level launch shapes of the star and transfer
        kernels, timed on this hierarchy (overwrites its work blocks)."""
        r = abi.mg_tune_report()
        check(lib.mg_autotune(self.h, reps, _stream(stream), C.byref(r)), "mg_autotune")
        return self._tune_dict(r)

    def autotune_solve(self, reps: int = 3, stream=None) -> dict:
        """mg_autotune_solve: the same shapes chosen by the time of whole FMG
        solves on this hierarchy's right-hand sides (times in us per solve)."""
        r = abi.mg_tune_report()
        check(lib.mg_autotune_solve(self.h, reps, _stream(stream), C.byref(r)), "mg_autotune_solve")
        return self._tune_dict(r)

    @staticmethod
    def _tune_dict(r) -> dict:
        out = {}
        for j in range(r.first_level, r.last_level + 1):
            out[j] = {"star_rows": r.star_rows[j] or "default",
                      "star_us": round(r.star_us[j], 2),
                      "star_default_us": round(r.star_default_us[j], 2)}
            if j >= 2:
                out[j].update({"transfer_rows": r.transfer_rows[j] or "default",
                               "transfer_us": round(r.transfer_us[j], 2),
                               "transfer_default_us": round(r.transfer_default_us[j], 2)})
        return out


class FP64MG:
    """The FP64 multigrid comparator (fp64_mg_* calls) for a BFP schedule:
    same shape, cycle, N and Chebyshev coefficients."""

    def __init__(self, params: abi.mg_params, device="cuda", stream=None):
        self.params = params
        nbytes = lib.fp64_mg_bytes(params.ndim, params.L)
        if nbytes == 0:
            raise BFPError(abi.BFP_EINVAL, "fp64_mg_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.arena.data_ptr()) % 256
        self.arena = self.arena[off:off + nbytes]
        c1 = params.c1.m * 2.0 ** params.c1.exp
        c2 = params.c2.m * 2.0 ** params.c2.exp
        h = C.c_void_p()
        check(lib.fp64_mg_create(params.ndim, params.L, params.nu1, params.nu2, params.N, c1, c2,
                                 _ptr(self.arena), nbytes, _stream(stream), C.byref(h)),
              "fp64_mg_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and lib is not None:
            lib.fp64_mg_destroy(h)
            self.h = None

    def fmg(self, rhs: list, out: torch.Tensor, stream=None) -> torch.Tensor:
        L = self.params.L
        if len(rhs) != L:
            raise ValueError(f"need {L} right-hand sides, got {len(rhs)}")
        side = (1 << L) + 1
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != side ** self.params.ndim:
            raise ValueError("out must be a contiguous float64 tensor of the padded finest grid")
        for j, f in enumerate(rhs, start=1):
            if f.dtype != torch.float64 or not f.is_contiguous() or f.numel() != ((1 << j) + 1) ** self.params.ndim:
                raise ValueError(f"rhs[{j - 1}] must hold the padded level-{j} grid in float64")
        self._ptrs = (C.c_void_p * L)(*[f.data_ptr() for f in rhs])
        check(lib.fp64_mg_fmg(self.h, self._ptrs, _ptr(out), _stream(stream)), "fp64_mg_fmg")
        return out


class Batch:
    """Independent problems solved together (mg_batch_* calls): one arena,
    one launch per batched solve."""

    def __init__(self, params: list, device="cuda", stream=None):
        self.params = list(params)
        arr = (abi.mg_params * len(self.params))(*self.params)
        self._arr = arr
        nbytes = lib.mg_batch_bytes(arr, len(self.params))
        if nbytes == 0:
            raise BFPError(abi.BFP_EINVAL, "mg_batch_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self.arena = self.arena[off:off + nbytes]
        b = C.c_void_p()
        check(lib.mg_batch_create(arr, len(self.params), _ptr(self.arena), nbytes,
                                  _stream(stream), C.byref(b)), "mg_batch_create")
        self.b = b

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value and lib is not None:
            lib.mg_batch_destroy(b)
            self.b = None

    def solve(self, rhs_table: torch.Tensor, stream=None) -> None:
        """rhs_table: int64 device tensor of len(params) * MG_MAX_LEVELS FP64
        device pointers (row i, column j - 1: problem i's f on level j)."""
        if rhs_table.dtype != torch.int64 or not rhs_table.is_cuda:
            raise ValueError("rhs_table must be an int64 device tensor of pointers")
        if rhs_table.numel() < len(self.params) * abi.MG_MAX_LEVELS:
            raise ValueError("rhs_table is too short")
        check(lib.mg_solve_batch(self.b, _ptr(rhs_table), _stream(stream)), "mg_solve_batch")

    def get_vec(self, prob: int, level: int, which: int = 0) -> Vec:
        v = abi.bfp_vec()
        check(lib.mg_batch_get_vec(self.b, prob, level, which, C.byref(v)), "mg_batch_get_vec")
        return Vec.view(v, self)

    def counters(self) -> tuple[float, int]:
        b = C.c_double()
        n = C.c_int64()
        check(lib.mg_batch_counters(self.b, C.byref(b), C.byref(n)), "mg_batch_counters")
        return b.value, n.value


class Server:
    """A request server in a torch-allocated arena of `budget` bytes
    (mg_server_* calls). submit() returns a ticket; poll() never blocks."""

    def __init__(self, budget: int, max_slots: int = 8, max_queue: int = 1 << 20,
                 exec_max_points: int = 0, device="cuda"):
        self.arena = torch.empty(budget + 256, dtype=torch.uint8, device=device)
        off = (-self.arena.data_ptr()) % 256
        self.arena = self.arena[off:off + budget]
        cfg = abi.mg_server_cfg(max_slots, max_queue, exec_max_points)
        s = C.c_void_p()
        check(lib.mg_server_create(C.byref(cfg), _ptr(self.arena), budget, C.byref(s)),
              "mg_server_create")
        self.s = s

    def __del__(self):
        s = getattr(self, "s", None)
        if s is not None and s.value and lib is not None:
            lib.mg_server_destroy(s)
            self.s = None

    def submit(self, params: abi.mg_params, rhs: list, x_out: torch.Tensor) -> int:
        """rhs[j - 1]: contiguous FP64 device tensor of f on level j (kept
        alive by the caller until the request is done); x_out: FP64 device
        tensor of (2^L + 1)^ndim values."""
        req = abi.mg_request()
        req.prm = params
        for j, f in enumerate(rhs):
            if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous():
                raise ValueError("rhs entries must be contiguous float64 device tensors")
            req.rhs_dev[j] = f.data_ptr()
        req.x_out_dev = x_out.data_ptr()
        t = C.c_uint64()
        check(lib.mg_server_submit(self.s, C.byref(req), C.byref(t)), "mg_server_submit")
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (status, gpu_ms)."""
        r = abi.mg_result()
        rc = lib.mg_server_poll(self.s, ticket, C.byref(r))
        if rc == abi.BFP_PENDING:
            return None
        check(rc, "mg_server_poll")
        return r.status, r.gpu_ms

    def collect(self, cap: int = 256) -> list:
        """Finished requests since the last call: [(ticket, status, gpu_ms)]."""
        if not hasattr(self, "_ct") or len(self._ct) < cap:
            self._ct = (C.c_uint64 * cap)()
            self._cr = (abi.mg_result * cap)()
        n = C.c_int()
        check(lib.mg_server_collect(self.s, self._ct, self._cr, cap, C.byref(n)),
              "mg_server_collect")
        return [(self._ct[i], self._cr[i].status, self._cr[i].gpu_ms) for i in range(n.value)]

    def stats(self) -> tuple[int, int, int]:
        q, r, b = C.c_int(), C.c_int(), C.c_size_t()
        check(lib.mg_server_stats(self.s, C.byref(q), C.byref(r), C.byref(b)), "mg_server_stats")
        return q.value, r.value, b.value


def mg_params_init(ndim: int, L: int, w: int, progressive: bool = True, nu1: int = 1,
                   nu2: int = 0, N: int = 2, policy: int = MG_POLICY_NN_IR_FIRST_Q,
                   eta_percent: int = 23, min_storage_bits: int = 0) -> abi.mg_params:
    p = abi.mg_params()
    check(lib.mg_params_init(ndim, L, w, int(progressive), nu1, nu2, N, policy, eta_percent,
                             C.byref(p)), "mg_params_init")
    p.min_storage_bits = min_storage_bits
    return p


def make_params(ndim: int, L: int, w_check: dict, w_work: dict, w_inner: dict,
                c1: abi.bfp_scalar, c2: abi.bfp_scalar, c1_gamma: abi.bfp_scalar,
                nu1: int = 1, nu2: int = 0, N: int = 2, policy: int = MG_POLICY_NN_IR_FIRST_Q,
                min_storage_bits: int = 0) -> abi.mg_params:
    p = abi.mg_params()
    p.ndim, p.L, p.nu1, p.nu2, p.N, p.policy = ndim, L, nu1, nu2, N, policy
    p.min_storage_bits = min_storage_bits
    for j in range(1, L + 1):
        p.w_check[j] = w_check[j]
        p.w_work[j] = w_work[j]
        p.w_inner[j] = w_inner[j]
    p.c1, p.c2, p.c1_gamma = c1, c2, c1_gamma
    return p


def batch_params(ndim: int, L: int, w_inner: int = 16, nu1: int = 1, nu2: int = 0,
                 N: int | None = None, policy: int = MG_POLICY_NN_IR_FIRST_Q,
                 eta_percent: int = 23) -> abi.mg_params:
    """Parameters of the batched workload: A and b at 32 bits, working width
    min(32, 2j + 8), inner width min(working, w_inner) on every level. With a
    fixed inner width the V-cycle's correction is only that accurate, so
    reaching the discretization error takes more IR iterations per level as
    the grid grows: N = max(2, L - 3) by default (2 up to 65^2, 4 at 129^2,
    5 at 257^2 for w_inner = 16)."""
    if N is None:
        N = max(2, L - 3)
    p = mg_params_init(ndim, L, w_inner, True, nu1, nu2, N, policy, eta_percent)
    for j in range(1, L + 1):
        p.w_check[j] = 32
        p.w_inner[j] = min(p.w_work[j], w_inner)
    return p
