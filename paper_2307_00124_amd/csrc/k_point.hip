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

template <typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_point(const PointLaunch L) {
  const int64_t n = L.n;
  const int64_t nchunk = (n + 2 + 1023) / 1024;
  const int64_t rr = interior_row(blockIdx.x / nchunk, n, L.ndim);
  const int64_t c = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  Epi<PASS, HASY> E;
  E.init(L.op);
  if (c < n + 2) {
    int32_t xv[4], yv[4] = {0, 0, 0, 0};
    ld4(X, rr * L.px + c, xv, true);
    if (HASY) ld4(Y, rr * L.py + c, yv, true);
    int64_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = E.apply(xv[k], yv[k]);
    if (PASS != kQ1) st4(Z, rr * L.pz + c, out);
  }
  E.finish();
}

template <typename TX, typename TY, typename TZ, int PASS, bool HASY>
static hipError_t point_go(const PointLaunch& L, hipStream_t s) {
  const int64_t rows = L.ndim == 3 ? L.n * L.n : L.n;
  const int64_t blocks = rows * ((L.n + 2 + 1023) / 1024);
  hipLaunchKernelGGL((k_point<TX, TY, TZ, PASS, HASY>), dim3((unsigned)blocks), dim3(kBlock), 0,
                     s, L);
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
  const int64_t n = L.n, side = n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t rr = interior_row(blockIdx.x / nchunk, n, L.ndim);
  const int64_t c0 = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  int64_t best = INT64_MIN;
  bool bad = false;
  for (int k = 0; k < 4; ++k) {
    const int64_t c = c0 + k;
    if (c < 1 || c > n) continue;
    int64_t z, e;
    bool fin;
    if (f64_parts(L.src[rr * side + c], z, e, fin)) {
      const int64_t nu = msb64(z) + e;
      best = nu > best ? nu : best;
    }
    bad |= !fin;
  }
  if (bad) atomicOr((unsigned long long*)&L.meta[kMetaFlags], 1ull);
  // block / grid max into the scratch slot; the last block publishes it
  __shared__ int64_t s_red[kBlock / 64];
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t b = s_red[0];
    for (int i = 1; i < kBlock / 64; ++i) b = s_red[i] > b ? s_red[i] : b;
    if (b != INT64_MIN) atomicMax((long long*)&L.meta[kMetaAccMax], (long long)b);
    __threadfence();
    unsigned long long t = atomicAdd((unsigned long long*)&L.meta[kMetaTicket], 1ull);
    if (t == (unsigned long long)gridDim.x - 1) {
      __threadfence();
      L.meta[kMetaMu] = atomic_load64(&L.meta[kMetaAccMax]);  // INT64_MIN: all zero
      atomic_store64(&L.meta[kMetaAccMax], INT64_MIN);
      atomic_store64(&L.meta[kMetaTicket], 0);
    }
  }
}

// pass 2: m_i = floor(x_i / 2^(max nu - w)), exponent max nu - w + log2_scale
template <typename T>
__global__ __launch_bounds__(kBlock) void k_f64_conv(const ConvertLaunch L) {
  const int64_t n = L.n, side = n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t rr = interior_row(blockIdx.x / nchunk, n, L.ndim);
  const int64_t c0 = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  const int64_t numax = L.meta[kMetaMu];
  const bool allzero = numax == INT64_MIN;
  const int64_t eq = allzero ? 1 - L.w : numax - L.w;     // exponent before scaling
  int64_t tmax = 0, tmin = 0;
  if (c0 < side) {
    int64_t out[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t c = c0 + k;
      out[k] = 0;
      if (c < 1 || c > n) continue;
      int64_t z, e;
      bool fin;
      if (f64_parts(L.src[rr * side + c], z, e, fin)) {
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

hipError_t launch_from_f64(const ConvertLaunch& L, hipStream_t s) {
  const int64_t rows = L.ndim == 3 ? L.n * L.n : L.n;
  const int64_t blocks = rows * ((L.n + 2 + 1023) / 1024);
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
  const int64_t side = L.n + 2;
  const int64_t nchunk = (side + 1023) / 1024;
  const int64_t row = blockIdx.x / nchunk;                 // every row, ring included
  const int64_t c0 = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  const int e = (int)L.meta[kMetaExp];
  const T* M = static_cast<const T*>(L.mant);
  for (int k = 0; k < 4; ++k) {
    const int64_t c = c0 + k;
    if (c < side) L.dst[row * side + c] = ldexp((double)M[row * L.pitch + c], e);
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
  if (i == kMetaAccMax) v = INT64_MIN;
  else if (i == kMetaAccMin) v = INT64_MAX;
  else if (i < 8) {
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
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(64), 0, s, meta, exp, 1);
  return hipGetLastError();
}

hipError_t launch_meta_reset(int64_t* meta, hipStream_t s) {
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(64), 0, s, meta, (int64_t)0, 0);
  return hipGetLastError();
}

// --------------------------------------------------------- exact dot ---

template <typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_dot(const DotLaunch L) {
  const int64_t n = L.n;
  const int64_t nchunk = (n + 2 + 1023) / 1024;
  const int64_t rr = interior_row(blockIdx.x / nchunk, n, L.ndim);
  const int64_t c = (int64_t)(blockIdx.x % nchunk) * 1024 + threadIdx.x * 4;
  __int128 acc = 0;
  if (c < n + 2) {
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
    int64_t* o = L.out;
    atomicAdd((unsigned long long*)&o[3], (unsigned long long)b0);
    atomicAdd((unsigned long long*)&o[4], (unsigned long long)b1);
    atomicAdd((unsigned long long*)&o[5], (unsigned long long)b2);
    __threadfence();
    unsigned long long t = atomicAdd((unsigned long long*)&o[6], 1ull);
    if (t == (unsigned long long)gridDim.x - 1) {
      __threadfence();
      const __int128 v = (__int128)(unsigned __int128)(uint64_t)atomic_load64(&o[3]) +
                         ((__int128)(unsigned __int128)(uint64_t)atomic_load64(&o[4]) << 32) +
                         ((__int128)atomic_load64(&o[5]) << 64);
      o[0] = (int64_t)(uint64_t)(unsigned __int128)v;
      o[1] = (int64_t)(v >> 64);
      o[2] = L.x_meta[kMetaExp] + L.y_meta[kMetaExp];
      atomic_store64(&o[3], 0);
      atomic_store64(&o[4], 0);
      atomic_store64(&o[5], 0);
      atomic_store64(&o[6], 0);
    }
  }
}

hipError_t launch_dot(const DotLaunch& L, hipStream_t s) {
  const int64_t rows = L.ndim == 3 ? L.n * L.n : L.n;
  const int64_t blocks = rows * ((L.n + 2 + 1023) / 1024);
  return with_type(L.xbits, [&](auto tx) {
    return with_type(L.ybits, [&](auto ty) {
      hipLaunchKernelGGL((k_dot<decltype(tx), decltype(ty)>), dim3((unsigned)blocks), dim3(kBlock),
                         0, s, L);
      return hipGetLastError();
    });
  });
}

}  // namespace bfpk
