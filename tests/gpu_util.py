"""Helpers of the GPU parity tests: move oracle blocks onto the device through
the library (bfp_vec_assign), read device blocks back, compare bit for bit."""
from __future__ import annotations

import numpy as np
import torch

import paper_2307_00124_amd as P
from oracle.bfp import BFP, as_block

DT = {8: torch.int8, 16: torch.int16, 32: torch.int32}


def upload(b: BFP, storage_bits: int | None = None) -> P.Vec:
    """Device copy of an oracle block (padded cubic layout, ring zero)."""
    side = b.m.shape[0]
    ndim = b.m.ndim
    v = P.Vec(ndim, side - 2, b.w, storage_bits)
    host = np.asarray(b.m.astype(np.int64), dtype=np.int64)
    v.mantissas().copy_(torch.from_numpy(host).to(DT[v.storage_bits]).cuda())
    P.bfp_vec_assign(v, b.e)
    return v


def download(v: P.Vec) -> tuple[int, np.ndarray, list]:
    torch.cuda.synchronize()
    meta = v.host_meta()
    m = v.mantissas().cpu().numpy().astype(np.int64)
    pad = v.padding()
    assert pad.numel() == 0 or int(pad.abs().max()) == 0, "row padding must stay zero"
    return meta[P.BFP_META_EXP], m, meta


def assert_block_equal(v: P.Vec, ref: BFP, what: str = "") -> None:
    e, m, meta = download(v)
    refm = np.asarray(ref.m.astype(np.int64), dtype=np.int64)
    bad = np.argwhere(m != refm)
    assert bad.size == 0, (f"{what}: {len(bad)} mantissas differ, first at {bad[0].tolist()}: "
                           f"gpu {m[tuple(bad[0])]} oracle {refm[tuple(bad[0])]}")
    assert e == ref.e, f"{what}: exponent gpu {e} oracle {ref.e}"
    assert meta[P.BFP_META_MAX] == max(0, int(refm.max())), what
    assert meta[P.BFP_META_MIN] == min(0, int(refm.min())), what


def rand_block(g: np.random.Generator, ndim: int, n: int, w: int, e: int,
               scale_bits: int | None = None) -> BFP:
    """Random mantissas in X_w (optionally only scale_bits wide) with a zero
    ring; several special patterns mixed in."""
    shape = (n + 2,) * ndim
    wb = scale_bits or w
    lo, hi = -(1 << (wb - 1)), (1 << (wb - 1)) - 1
    m = g.integers(lo, hi, size=shape, endpoint=True, dtype=np.int64)
    flat = m.reshape(-1)
    k = max(1, flat.size // 50)
    idx = g.integers(0, flat.size, k)
    flat[idx[: k // 3]] = lo
    flat[idx[k // 3: 2 * k // 3]] = hi
    flat[idx[2 * k // 3:]] = 0
    inner = np.zeros(shape, dtype=bool)
    inner[(slice(1, -1),) * ndim] = True
    m[~inner] = 0
    return BFP(e, as_block(m), w)
