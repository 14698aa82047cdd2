"""The C-ABI library loads, exports what include/bfpmg.h declares, and its
host-only entry points (layout, schedules, Chebyshev coefficients, argument
validation) behave — no device work is started here."""
import ctypes as C
import os
import re
from fractions import Fraction

import pytest

import paper_2307_00124_amd as P
from paper_2307_00124_amd import abi
from oracle import mg

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "bfpmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("bfp_", "mg_"))))


def test_every_declared_function_is_exported_and_bound():
    names = declared_functions()
    assert len(names) >= 25
    lib = C.CDLL(abi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
        assert n in abi.SIGNATURES, f"{n} has no ctypes signature"


def test_header_constants_match_the_binding_and_the_oracle():
    text = open(HEADER).read()
    macros = dict(re.findall(r"^#define\s+(\w+)\s+(\d+)\s*$", text, flags=re.M))
    for name in ("MG_MAX_LEVELS", "MG_DIAG_SITES", "MG_DIAG_BINS", "MG_DIAG_GAP_BINS"):
        assert int(macros[name]) == getattr(abi, name), name
    assert abi.MG_DIAG_SITES == len(mg.SITES)
    assert abi.MG_DIAG_BINS == mg.DIAG_BINS and abi.MG_DIAG_GAP_BINS == mg.DIAG_GAP_BINS


def test_layout():
    assert P.bfp_layout(2, 4095, 32) == (4128, 4128 * 4097 * 4)
    assert P.bfp_layout(2, 31, 16) == (64, 64 * 33 * 2)
    assert P.bfp_layout(3, 511, 8) == (640, 640 * 513 * 513)
    assert P.bfp_layout(2, 30, 32) == (32, 32 * 32 * 4)
    with pytest.raises(P.BFPError):
        P.bfp_layout(4, 7, 32)
    with pytest.raises(P.BFPError):
        P.bfp_layout(2, 7, 12)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("eta", [1, 13, 23, 50, 99])
def test_cheby_coefficients_match_oracle(ndim, eta):
    p = P.mg_params_init(ndim, 5, 24, eta_percent=eta)
    sm = mg.make_smoother(ndim, Fraction(eta, 100))
    assert (p.c1.m, p.c1.exp) == (sm.c1.m, sm.c1.e)
    assert (p.c2.m, p.c2.exp) == (sm.c2.m, sm.c2.e)
    assert (p.c1_gamma.m, p.c1_gamma.exp) == (sm.c1_gamma.m, sm.c1_gamma.e)


@pytest.mark.parametrize("L,w", [(5, 8), (9, 16), (12, 24), (12, 32), (7, 5)])
def test_progressive_schedule_matches_oracle(L, w):
    p = P.mg_params_init(2, L, w, progressive=True)
    s = mg.widths_progressive(L, w)
    for j in range(1, L + 1):
        assert (p.w_check[j], p.w_work[j], p.w_inner[j]) == (s.check[j], s.work[j], s.inner[j])
    f = P.mg_params_init(2, L, w, progressive=False)
    assert all(f.w_inner[j] == f.w_work[j] == f.w_check[j] == w for j in range(1, L + 1))


def test_hierarchy_size_is_host_computable():
    p = P.mg_params_init(2, 12, 16)
    nbytes = P.lib.mg_hierarchy_bytes(C.byref(p))
    assert 300e6 < nbytes < 600e6
    bad = P.mg_params_init(2, 5, 16)
    bad.nu1 = 0
    assert P.lib.mg_hierarchy_bytes(C.byref(bad)) == 0


def _fake_vec(n=7, w=16, bits=16, ndim=2):
    pitch, _ = P.bfp_layout(ndim, n, bits)
    return abi.bfp_vec(0x10000, 0x20000, w, bits, ndim, n, pitch)


def test_validation_errors_before_any_launch():
    A = P.Stencil(2, P.BFP_STENCIL_A, -2, [0, -1, 0, -1, 4, -1, 0, -1, 0]).c()
    x, z = _fake_vec(), _fake_vec()
    z.mant, z.meta = 0x30000, 0x40000
    one = P.scalar(1, 0)
    g = P.gamma_explicit(1, 0)
    lib = P.lib
    # width beyond storage
    rc = lib.bfp_stencil_apply(C.byref(A), C.byref(x), C.byref(one), None, None, 17,
                               P.BFP_SATURATE, C.byref(g), C.byref(z), None)
    assert rc == abi.BFP_EWIDTH
    # aliasing input and output of a stencil
    rc = lib.bfp_stencil_apply(C.byref(A), C.byref(x), C.byref(one), None, None, 8,
                               P.BFP_SATURATE, C.byref(g), C.byref(x), None)
    assert rc == abi.BFP_EINVAL
    # shape mismatch
    z2 = _fake_vec(n=9)
    z2.mant, z2.meta = 0x30000, 0x40000
    rc = lib.bfp_stencil_apply(C.byref(A), C.byref(x), C.byref(one), None, None, 8,
                               P.BFP_SATURATE, C.byref(g), C.byref(z2), None)
    assert rc == abi.BFP_ESHAPE
    # saturate mode without an estimate
    rc = lib.bfp_stencil_apply(C.byref(A), C.byref(x), C.byref(one), None, None, 8,
                               P.BFP_SATURATE, None, C.byref(z), None)
    assert rc == abi.BFP_EINVAL
    # exact budget: a 32-bit alpha times a 32-bit stencil input
    x32 = _fake_vec(w=32, bits=32)
    z32 = _fake_vec(w=32, bits=32)
    z32.mant, z32.meta = 0x30000, 0x40000
    big = P.scalar(-(1 << 31), 0, 32)
    rc = lib.bfp_stencil_apply(C.byref(A), C.byref(x32), C.byref(big), None, None, 8,
                               P.BFP_SATURATE, C.byref(g), C.byref(z32), None)
    assert rc == abi.BFP_EWIDTH
    assert b"budget" in lib.bfp_last_error()
    # non-star same-grid stencil
    B = P.Stencil(2, P.BFP_STENCIL_A, -2, [1, -1, 0, -1, 4, -1, 0, -1, 0]).c()
    rc = lib.bfp_stencil_apply(C.byref(B), C.byref(x), C.byref(one), None, None, 8,
                               P.BFP_SATURATE, C.byref(g), C.byref(z), None)
    assert rc == abi.BFP_EINVAL
    # transfer sizes must nest
    R = P.Stencil(2, P.BFP_STENCIL_R, -2, [1, 2, 1, 2, 4, 2, 1, 2, 1]).c()
    zc = _fake_vec(n=4)
    zc.mant, zc.meta = 0x30000, 0x40000
    rc = lib.bfp_stencil_apply(C.byref(R), C.byref(x), C.byref(one), None, None, 8,
                               P.BFP_SATURATE, C.byref(g), C.byref(zc), None)
    assert rc == abi.BFP_ESHAPE


def test_cheby_argument_errors():
    c1, c2 = abi.bfp_scalar(), abi.bfp_scalar()
    assert P.lib.bfp_cheby_coeffs(2, 1, 100, 100, 1, 1, 16, C.byref(c1), C.byref(c2)) == abi.BFP_EINVAL
    assert P.lib.bfp_cheby_coeffs(2, 1, 23, 100, 1, 1, 40, C.byref(c1), C.byref(c2)) == abi.BFP_EWIDTH


def test_tuning_keys_and_autotuner_arguments():
    """The tuning keys of the optional fused relaxation + residual and of the
    one-launch finite-element ops round-trip and range-check; the autotuners reject a missing hierarchy (host-side
    checks, no launch)."""
    lib = P.lib
    v = C.c_int()
    for key, val in (("fuse_relax_res", 1), ("relax_res_rows", 8), ("relax_res_max_n", 511),
                     ("fe_one_launch", 0), ("fe_program", 0)):
        old = C.c_int()
        assert lib.bfp_tuning_get(key.encode(), C.byref(old)) == abi.BFP_OK
        assert lib.bfp_tuning_set(key.encode(), val) == abi.BFP_OK
        assert lib.bfp_tuning_get(key.encode(), C.byref(v)) == abi.BFP_OK and v.value == val
        assert lib.bfp_tuning_set(key.encode(), old.value) == abi.BFP_OK
    assert lib.bfp_tuning_set(b"fuse_relax_res", 2) == abi.BFP_EINVAL
    assert lib.bfp_tuning_set(b"relax_res_rows", 2000) == abi.BFP_EINVAL
    assert lib.bfp_tuning_set(b"fe_one_launch", 4097) == abi.BFP_EINVAL
    assert lib.bfp_tuning_set(b"fe_program", 2) == abi.BFP_EINVAL
    assert lib.bfp_tuning_get(b"fuse_relax_res", C.byref(v)) == abi.BFP_OK and v.value == 0
    assert lib.bfp_tuning_get(b"fe_one_launch", C.byref(v)) == abi.BFP_OK and v.value == 4096
    r = abi.mg_tune_report()
    assert lib.mg_autotune_solve(None, 3, None, C.byref(r)) == abi.BFP_EINVAL
    assert lib.mg_autotune(None, 3, None, C.byref(r)) == abi.BFP_EINVAL


def test_stream_copy_argument_errors():
    """bfp_stream_copy checks size, alignment and pointers on the host."""
    lib = P.lib
    assert lib.bfp_stream_copy(None, None, 0, 0, None) == abi.BFP_OK
    assert lib.bfp_stream_copy(0x1000, 0x2000, 24, 0, None) == abi.BFP_EINVAL
    assert lib.bfp_stream_copy(0x1008, 0x2000, 32, 0, None) == abi.BFP_EINVAL
    assert lib.bfp_stream_copy(None, 0x2000, 32, 0, None) == abi.BFP_EINVAL
    assert lib.bfp_stream_copy(0x1000, 0x2000, 32, 2, None) == abi.BFP_EINVAL
    assert lib.bfp_stream_copy(0x1000, 0x2000, -16, 0, None) == abi.BFP_EINVAL
