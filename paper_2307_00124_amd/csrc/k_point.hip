// Pointwise BFP kernels: axpby / sub / normalize / saturate-truncate through
// the common epilogue, FP64 <-> BFP conversion, block initialisation and the
// exact dot product.
//
// Every kernel walks the interior rows of the padded, row-pitched grid; a
// block covers 1024 columns of one row (4 per thread). Ring and padding
// entries are zero in every block and stay zero.
#include "epilogue.hpp"

namespace bfpk {

__device__ __forceinline__ int64_t interior_row(int64_t row, int64_t n, int nd) {
  return nd == 3 ? (row / n + 1) * (n + 2) + (row % n + 1) : row + 1;
}

// work items: (interior row, 1024-column chunk) pairs, grid-strided
__host__ __device__ inline int64_t row_items(int64_t n, int ndim) {
  return (ndim == 3 ? n * n : n) * ((n + 2 + 1023) / 1024);
}
inline unsigned grid_for(int64_t items) {
  return (unsigned)(items < kMaxBlocks ? items : kMaxBlocks);
}

template <typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_point(const PointLaunch L) {
  const int64_t n = L.n;
  const int64_t nchunk = (n + 2 + 1023) / 1024;
  const int64_t items = row_items(n, L.ndim);
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  // kPU items per round, their loads issued before any of them is used (a
  // round keeps kPU times the bytes of one item in flight)
  constexpr int kPU = 4;
  int32_t xv[kPU][4], yv[kPU][4];
  int64_t rr[kPU], c[kPU];
  bool live[kPU];
  auto fetch = [&](int64_t it0) {
#pragma unroll
    for (int u = 0; u < kPU; ++u) {
      const int64_t it = it0 + (int64_t)u * gridDim.x;
      rr[u] = interior_row((it < items ? it : 0) / nchunk, n, L.ndim);
      c[u] = ((it < items ? it : 0) % nchunk) * 1024 + threadIdx.x * 4;
      live[u] = it < items && c[u] < n + 2;
      ld4(X, rr[u] * L.px + c[u], xv[u], live[u]);
      if (HASY) ld4(Y, rr[u] * L.py + c[u], yv[u], live[u]);
      else yv[u][0] = yv[u][1] = yv[u][2] = yv[u][3] = 0;
    }
  };
  // the first round's loads are issued before the epilogue reads the
  // operands' metadata (they do not depend on it), so the round trips overlap
  fetch(blockIdx.x);
  Epi<PASS, HASY> E;
  E.init(L.op);
  with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    for (int64_t it0 = blockIdx.x; it0 < items; it0 += (int64_t)kPU * gridDim.x) {
      if (it0 != blockIdx.x) fetch(it0);
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        if (!live[u]) continue;
        int64_t out[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = E.template put<VAR>(xv[u][k], yv[u][k], true);
        if (PASS != kQ1) st4(Z, rr[u] * L.pz + c[u], out);
      }
    }
  });
  E.finish();
}

template <typename TX, typename TY, typename TZ, int PASS, bool HASY>
static hipError_t point_go(const PointLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_point<TX, TY, TZ, PASS, HASY>), dim3(grid_for(row_items(L.n, L.ndim))),
                     dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

hipError_t launch_point(const PointLaunch& L, hipStream_t s) {
  const bool q1 = L.op.mode == kModeQ1;
  return with_type(L.xbits, [&](auto tx) {
    using TX = decltype(tx);
    if (!L.op.has_y) {
      if (q1) return point_go<TX, int32_t, int32_t, kQ1, false>(L, s);
      return with_type(L.zbits, [&](auto tz) {
        return point_go<TX, int32_t, decltype(tz), kOut, false>(L, s);
      });
    }
    return with_type(L.ybits, [&](auto ty) {
      using TY = decltype(ty);
      if (q1) return point_go<TX, TY, int32_t, kQ1, true>(L, s);
      return with_type(L.zbits, [&](auto tz) {
        return point_go<TX, TY, decltype(tz), kOut, true>(L, s);
      });
    });
  });
}

// ------------------------------------------------------- FP64 -> BFP ----

// Decompose a finite double as z * 2^e with integer z (|z| < 2^53).
__device__ __forceinline__ bool f64_parts(double x, int64_t& z, int64_t& e, bool& finite) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int64_t E = (int64_t)((b >> 52) & 0x7FF);
  const int64_t F = (int64_t)(b & ((1ull << 52) - 1));
  finite = E != 0x7FF;
  if (!finite || (E == 0 && F == 0)) return false;
  const int64_t M = E ? (F | (1ll << 52)) : F;
  e = E ? E - 1075 : -1074;
  z = (b >> 63) ? -M : M;
  return true;
}

// pass 1: max_i nu(x_i) over the interior, and the non-finite flag
__global__ __launch_bounds__(kBlock) void k_f64_nu(const ConvertLaunch L) {
  const double* src = L.src ? L.src : L.src_table[L.table_index];
  const int64_t n = L.n, side = n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t items = row_items(n, L.ndim);
  int64_t best = INT64_MIN;
  bool bad = false;
  auto take = [&](double x) {
    int64_t z, e;
    bool fin;
    if (f64_parts(x, z, e, fin)) {
      const int64_t nu = msb64(z) + e;
      best = nu > best ? nu : best;
    }
    bad |= !fin;
  };
  // 16-byte loads: a row starting at an odd element (rows alternate, the
  // row length n + 2 being odd) is read in pairs shifted by one column, so
  // every pair is aligned; each interior column still lies in exactly one
  // thread's four columns, and a pair is read only when both of its
  // columns lie in the row
  const bool al16 = ((uintptr_t)src & 15) == 0;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t rr = interior_row(it / nchunk, n, L.ndim);
    const int64_t c0 = (it % nchunk) * 1024 + threadIdx.x * 4;
    const int64_t g0 = rr * side;
    if (al16) {
      const int64_t cs = c0 - (g0 & 1);
      double v[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t p = cs + 2 * h;
        const bool ok = p >= 0 && p + 1 <= n + 1;
        const double2 q = *reinterpret_cast<const double2*>(src + (ok ? g0 + p : 0));
        v[2 * h] = ok ? q.x : 0.0;
        v[2 * h + 1] = ok ? q.y : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t c = cs + k;
        if (c >= 1 && c <= n) take(v[k]);
      }
    } else {
      for (int k = 0; k < 4; ++k) {
        const int64_t c = c0 + k;
        if (c >= 1 && c <= n) take(src[g0 + c]);
      }
    }
  }
  if (bad) atomicOr((unsigned long long*)&L.meta[kMetaFlags], 1ull);
  // grid max of nu into the accumulator sets; the last block publishes it
  // in kMetaMu (INT64_MIN when every value is zero)
  __shared__ int64_t s_red[kBlock / 64];
  const int64_t b = block_max(best, s_red);
  if (threadIdx.x == 0) {
    int64_t* set = acc_set(L.meta);
    if (take_ticket(L.meta, amax(&set[kAccMax], b))) {
      int64_t mx = INT64_MIN;
      for (int k = 0; k < kSets; ++k) {
        const int64_t a = axch(&L.meta[kSetBase + kSetStride * k + kAccMax], INT64_MIN);
        mx = a > mx ? a : mx;
      }
      axch(&L.meta[kMetaTicket], 0);
      L.meta[kMetaMu] = mx;
    }
  }
}

// pass 2: m_i = floor(x_i / 2^(max nu - w)), exponent max nu - w + log2_scale
template <typename T>
__global__ __launch_bounds__(kBlock) void k_f64_conv(const ConvertLaunch L) {
  const double* src = L.src ? L.src : L.src_table[L.table_index];
  const int64_t n = L.n, side = n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t items = row_items(n, L.ndim);
  const int64_t numax = L.meta[kMetaMu];
  const bool allzero = numax == INT64_MIN;
  const int64_t eq = allzero ? 1 - L.w : numax - L.w;     // exponent before scaling
  int64_t tmax = 0, tmin = 0;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t rr = interior_row(it / nchunk, n, L.ndim);
    const int64_t c0 = (it % nchunk) * 1024 + threadIdx.x * 4;
    if (c0 >= side) continue;
    int64_t out[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t c = c0 + k;
      out[k] = 0;
      if (c < 1 || c > n) continue;
      int64_t z, e;
      bool fin;
      if (f64_parts(src[rr * side + c], z, e, fin)) {
        const int64_t sh = e - eq;
        out[k] = sh >= 0 ? (int64_t)((uint64_t)z << sh) : shr_floor(z, -sh);
        tmax = out[k] > tmax ? out[k] : tmax;
        tmin = out[k] < tmin ? out[k] : tmin;
      }
    }
    st4(static_cast<T*>(L.mant), rr * L.pitch + c0, out);
  }
  finish_outputs(tmax, tmin, 0, L.meta, eq + L.log2_scale);
}

// ------------------------------------------------- streaming copy -------

// A plain device copy of 16-byte words, CU in flight per thread and
// grid-strided: the streaming-bandwidth reference the BFP kernels are
// measured against (NT: non-temporal loads and stores).
template <bool NT, int CU>
__global__ __launch_bounds__(kBlock) void k_stream_copy(const v4i32* __restrict__ src,
                                                      v4i32* __restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < n16; i0 += CU * stride) {
    v4i32 v[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int64_t i = i0 + u * stride;
      const v4i32* p = src + (i < n16 ? i : 0);
      v[u] = NT ? __builtin_nontemporal_load(p) : *p;
    }
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n16) {
        if (NT) __builtin_nontemporal_store(v[u], dst + i);
        else dst[i] = v[u];
      }
    }
  }
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, bool nontemporal,
                              int max_blocks, int per_thread, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int cu = per_thread >= 8 ? 8 : 4;
  const int64_t per_block = (int64_t)kBlock * cu;
  int64_t blocks = (n16 + per_block - 1) / per_block;
  if (blocks > max_blocks) blocks = max_blocks;
  const v4i32* a = static_cast<const v4i32*>(src);
  v4i32* b = static_cast<v4i32*>(dst);
  const dim3 g((unsigned)blocks), t(kBlock);
  if (nontemporal) {
    if (cu == 8) hipLaunchKernelGGL((k_stream_copy<true, 8>), g, t, 0, s, a, b, n16);
    else hipLaunchKernelGGL((k_stream_copy<true, 4>), g, t, 0, s, a, b, n16);
  } else {
    if (cu == 8) hipLaunchKernelGGL((k_stream_copy<false, 8>), g, t, 0, s, a, b, n16);
    else hipLaunchKernelGGL((k_stream_copy<false, 4>), g, t, 0, s, a, b, n16);
  }
  return hipGetLastError();
}

hipError_t launch_from_f64(const ConvertLaunch& L, hipStream_t s) {
  const unsigned blocks = grid_for(row_items(L.n, L.ndim));
  hipLaunchKernelGGL(k_f64_nu, dim3((unsigned)blocks), dim3(kBlock), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return with_type(L.bits, [&](auto t) {
    hipLaunchKernelGGL((k_f64_conv<decltype(t)>), dim3((unsigned)blocks), dim3(kBlock), 0, s, L);
    return hipGetLastError();
  });
}

// ------------------------------------------------------- BFP -> FP64 ----

template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_f64(const ConvertLaunch L) {
  double* dst = L.dst ? L.dst : L.dst_table[L.table_index];
  const int64_t side = L.n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t row = blockIdx.x / nchunk;                 // every row, ring included
  const int64_t c0 = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  const int e = (int)L.meta[kMetaExp];
  const T* M = static_cast<const T*>(L.mant);
  for (int k = 0; k < 4; ++k) {
    const int64_t c = c0 + k;
    if (c < side) dst[row * side + c] = ldexp((double)M[row * L.pitch + c], e);
  }
}

hipError_t launch_to_f64(const ConvertLaunch& L, hipStream_t s) {
  const int64_t side = L.n + 2;
  const int64_t rows = L.ndim == 3 ? side * side : side;
  const int64_t blocks = rows * ((side + 1023) / 1024);
  return with_type(L.bits, [&](auto t) {
    hipLaunchKernelGGL((k_to_f64<decltype(t)>), dim3((unsigned)blocks), dim3(kBlock), 0, s, L);
    return hipGetLastError();
  });
}

// ----------------------------------------------------- initialisation ---

__global__ __launch_bounds__(kBlock) void k_zero16(uint4* p, int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_meta_init(int64_t* m, int64_t exp, int full) {
  const int i = threadIdx.x;
  if (i >= kMetaSlots) return;
  int64_t v = 0;
  if (i >= kSetBase) {
    const int f = (i - kSetBase) % kSetStride;
    v = f == kAccMax ? INT64_MIN : (f == kAccMin ? INT64_MAX : 0);
  } else if (i < kMetaTicket) {
    if (!full) return;
    v = i == kMetaExp ? exp : (i == kMetaMu ? 1 : 0);
  }
  m[i] = v;
}

hipError_t launch_init(void* mant, size_t bytes, int64_t* meta, int64_t exp, hipStream_t s) {
  if (mant && bytes) {
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_zero16, dim3((unsigned)((n16 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, static_cast<uint4*>(mant), n16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(kMetaSlots), 0, s, meta, exp, 1);
  return hipGetLastError();
}

// one block per metadata block of a list: exponent exps[b], identities elsewhere
__global__ void k_meta_init_list(int64_t* const* metas, const int64_t* exps) {
  int64_t* m = metas[blockIdx.x];
  const int i = threadIdx.x;
  if (i >= kMetaSlots) return;
  int64_t v = 0;
  if (i >= kSetBase) {
    const int f = (i - kSetBase) % kSetStride;
    v = f == kAccMax ? INT64_MIN : (f == kAccMin ? INT64_MAX : 0);
  } else if (i < kMetaTicket) {
    v = i == kMetaExp ? exps[blockIdx.x] : (i == kMetaMu ? 1 : 0);
  }
  m[i] = v;
}

hipError_t launch_meta_init_list(int64_t* const* metas_dev, const int64_t* exps_dev, int count,
                                 hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_meta_init_list, dim3((unsigned)count), dim3(kMetaSlots), 0, s, metas_dev,
                     exps_dev);
  return hipGetLastError();
}

hipError_t launch_meta_reset(int64_t* meta, hipStream_t s) {
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(kMetaSlots), 0, s, meta, (int64_t)0, 0);
  return hipGetLastError();
}

// --------------------------------------------------------- exact dot ---

template <typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_dot(const DotLaunch L) {
  const int64_t n = L.n;
  const int64_t nchunk = (n + 2 + 1023) / 1024;
  const int64_t items = row_items(n, L.ndim);
  __int128 acc = 0;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t rr = interior_row(it / nchunk, n, L.ndim);
    const int64_t c = (it % nchunk) * 1024 + threadIdx.x * 4;
    if (c >= n + 2) continue;
    int32_t xv[4], yv[4];
    ld4(static_cast<const TX*>(L.x), rr * L.px + c, xv, true);
    ld4(static_cast<const TY*>(L.y), rr * L.py + c, yv, true);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += (__int128)((int64_t)xv[k] * (int64_t)yv[k]);
  }
  // split into limbs: l0, l1 unsigned 32-bit, l2 the signed high 64 bits
  const unsigned __int128 u = (unsigned __int128)acc;
  int64_t l0 = (int64_t)(uint32_t)u, l1 = (int64_t)(uint32_t)(u >> 32);
  int64_t l2 = (int64_t)(acc >> 64);
  l0 = wave_sum(l0);
  l1 = wave_sum(l1);
  l2 = wave_sum(l2);
  __shared__ int64_t s_red[3][kBlock / 64];
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = l0;
    s_red[1][threadIdx.x >> 6] = l1;
    s_red[2][threadIdx.x >> 6] = l2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t b0 = 0, b1 = 0, b2 = 0;
    for (int i = 0; i < kBlock / 64; ++i) { b0 += s_red[0][i]; b1 += s_red[1][i]; b2 += s_red[2][i]; }
    // limbs go to accumulator sets laid out like a block's metadata scratch
    int64_t* o = L.out;
    int64_t* set = acc_set(o);
    const int64_t r = aadd(&set[0], b0) ^ aadd(&set[1], b1) ^ aadd(&set[2], b2);
    if (take_ticket(o, r)) {
      __int128 v = 0;
      for (int k = 0; k < kSets; ++k) {
        int64_t* sk = o + kSetBase + kSetStride * k;
        v += (__int128)(unsigned __int128)(uint64_t)axch(&sk[0], 0);
        v += (__int128)(unsigned __int128)(uint64_t)axch(&sk[1], 0) << 32;
        v += (__int128)axch(&sk[2], 0) << 64;
      }
      axch(&o[kMetaTicket], 0);
      o[0] = (int64_t)(uint64_t)(unsigned __int128)v;
      o[1] = (int64_t)(v >> 64);
      o[2] = L.x_meta[kMetaExp] + L.y_meta[kMetaExp];
    }
  }
}

// Diagnostics of a launched operation (one thread each). Between the two
// qcomp passes, mu* (from the first) and the estimate's metadata (not yet
// changed by the second) give the window gap of the call; after an nnqcomp
// call, the output's saturation count.
__global__ void k_diag_q(const OpArgs op) {
  const Resolved r = resolve(op, ptr_meta(op));
  bool zero;
  const int64_t nu = gamma_nu(op.g, ptr_meta(op), &zero);
  // mu* = eo - ez + w_out in the second pass
  if (!zero) diag_count(op.diag, diag_gap_bin(nu - r.ez - (r.eo - r.ez + op.w_out)), 0, 0);
}

__global__ void k_diag_sat(int64_t* diag, const int64_t* zm) {
  diag_count(diag, -1, 1, zm[kMetaSat]);
}

hipError_t launch_diag_q(const OpArgs& op, hipStream_t s) {
  OpArgs o = op;
  o.mode = kModeQ2;
  hipLaunchKernelGGL(k_diag_q, dim3(1), dim3(1), 0, s, o);
  return hipGetLastError();
}

hipError_t launch_diag_sat(int64_t* diag, const int64_t* zm, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_sat, dim3(1), dim3(1), 0, s, diag, zm);
  return hipGetLastError();
}

hipError_t launch_dot(const DotLaunch& L, hipStream_t s) {
  const unsigned blocks = grid_for(row_items(L.n, L.ndim));
  return with_type(L.xbits, [&](auto tx) {
    return with_type(L.ybits, [&](auto ty) {
      hipLaunchKernelGGL((k_dot<decltype(tx), decltype(ty)>), dim3((unsigned)blocks), dim3(kBlock),
                         0, s, L);
      return hipGetLastError();
    });
  });
}

// ------------------------------------------------------- unit vector ---

// A zero block becomes the unit vector e_pos at w bits: the normalized
// floor quantization of 1.0 (nu(1) = 2, so e = 2 - w and m = 2^(w-2)).
__global__ void k_unit(void* mant, int bits, int64_t pos, int64_t* meta, int w) {
  if (threadIdx.x != 0) return;
  const int64_t m = (int64_t)1 << (w - 2);
  if (bits == 32) static_cast<int32_t*>(mant)[pos] = (int32_t)m;
  else if (bits == 16) static_cast<int16_t*>(mant)[pos] = (int16_t)m;
  else static_cast<int8_t*>(mant)[pos] = (int8_t)m;
  meta[kMetaExp] = 2 - w;
  meta[kMetaMax] = m;
  meta[kMetaMin] = 0;
  meta[kMetaSat] = 0;
}

hipError_t launch_unit(void* mant, int bits, int64_t pos, int64_t* meta, int w, hipStream_t s) {
  hipLaunchKernelGGL(k_unit, dim3(1), dim3(64), 0, s, mant, bits, pos, meta, w);
  return hipGetLastError();
}

}  // namespace bfpk
