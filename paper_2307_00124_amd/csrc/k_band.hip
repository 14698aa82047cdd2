// Banded BFP matrix-vector products on 1D blocks (the finite-element model
// problems): z = Q(alpha M x + beta y) with M a BFP matrix of one exponent
// whose row i holds `band` integer taps from input column col0[i] (the exact
// gemv / spmv rows of Appendix B), through the common epilogue. Vectors are
// padded 1D blocks (index 0 and n + 1 are the zero ends); an identity
// matrix (no taps) gives the pointwise axpby / sub rows.
#include "band.hpp"
#include "epilogue.hpp"

namespace bfpk {

template <int PASS, bool HASY, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_band(const BandLaunch L) {
  const int32_t* X = L.x;
  const int32_t* Y = L.y;
  Epi<PASS, HASY> E;
  E.init(L.op);
  with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < L.nout;
         i += (int64_t)gridDim.x * kBlock) {
      int64_t g = 0;
      if (IDENT) {
        g = X[1 + i];
      } else {
        const int32_t* t = L.taps + i * L.band;
        const int32_t* xr = X + 1 + L.col0[i];
        for (int k = 0; k < L.band; ++k) g += (int64_t)t[k] * xr[k];
      }
      const int32_t yv = HASY ? Y[1 + i] : 0;
      const int64_t out = E.template put<VAR>(g, yv, true);
      if (PASS != kQ1) L.z[1 + i] = (int32_t)out;
    }
  });
  E.finish();
}

// Both qcomp passes in one workgroup that holds every output point
// (nout <= U kBlock, point i on lane i mod kBlock): each lane keeps the
// exact terms of its U points in registers, the block's
// mu* = max(1, max msb z*_i) comes from an LDS reduction and feeds the
// second pass directly (it is also stored in the output's metadata, as the
// two-launch form does). Same arithmetic as k_band<kQ1> then k_band<kOut>.
// `base` reads the operands' metadata.
template <bool HASY, bool IDENT, int U, class MA>
__device__ __forceinline__ void band_qcomp_block(const BandLaunch& L, const MA& base) {
  int64_t g[U];
  int32_t yv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = (int)threadIdx.x + u * kBlock;
    g[u] = 0;
    yv[u] = 0;
    if (i < L.nout) {
      if (IDENT) {
        g[u] = L.x[1 + i];
      } else {
        const int32_t* t = L.taps + (int64_t)i * L.band;
        const int32_t* xr = L.x + 1 + L.col0[i];
        int64_t a = 0;
        for (int k = 0; k < L.band; ++k) a += (int64_t)t[k] * xr[k];
        g[u] = a;
      }
      if (HASY) yv[u] = L.y[1 + i];
    }
  }
  OpArgs op = L.op;
  op.mode = kModeQ1;
  Epi<kQ1, HASY> E1;
  E1.init(op, base);
  with_fast(E1, [&](auto fast_tag) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      E1.template put<decltype(fast_tag)::value>(g[u], yv[u],
                                                 (int)threadIdx.x + u * kBlock < L.nout);
  });
  // mu* (at most 127) and the outputs' max / min / saturation count fit
  // 32 bits: 32-bit wave reductions
  __shared__ int32_t s_mu[kBlock / 64];
  const int32_t wmu = wave_max32((int32_t)E1.tmu);
  if ((threadIdx.x & 63) == 0) s_mu[threadIdx.x >> 6] = wmu;
  __syncthreads();
  int64_t mu = 1;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) mu = s_mu[w] > mu ? s_mu[w] : mu;
  if (threadIdx.x == 0) op.z_meta[kMetaMu] = mu;
  op.mode = kModeQ2;
  auto ma = [&](int o, int k) -> int64_t { return o == kOpZ && k == kMetaMu ? mu : base(o, k); };
  Epi<kOut, HASY> E2;
  E2.init(op, ma);
  int32_t out[U];
  with_fast(E2, [&](auto fast_tag) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      out[u] = (int32_t)E2.template put<decltype(fast_tag)::value>(
          g[u], yv[u], (int)threadIdx.x + u * kBlock < L.nout);
  });
  {
    __shared__ int32_t s_red[3][kBlock / 64];
    const int32_t a = wave_max32(E2.tmax), b = wave_min32(E2.tmin), c = wave_sum32(E2.tsat);
    if ((threadIdx.x & 63) == 0) {
      s_red[0][threadIdx.x >> 6] = a;
      s_red[1][threadIdx.x >> 6] = b;
      s_red[2][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t bmax = s_red[0][0], bmin = s_red[1][0];
      int64_t bsat = s_red[2][0];
      for (int w = 1; w < kBlock / 64; ++w) {
        bmax = s_red[0][w] > bmax ? s_red[0][w] : bmax;
        bmin = s_red[1][w] < bmin ? s_red[1][w] : bmin;
        bsat += s_red[2][w];
      }
      op.z_meta[kMetaMax] = bmax;
      op.z_meta[kMetaMin] = bmin;
      op.z_meta[kMetaSat] = bsat;
      op.z_meta[kMetaExp] = E2.R.eo;
    }
  }
  // the outputs are stored after the reduction (measured faster than
  // storing them between the epilogue and the reduction)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = (int)threadIdx.x + u * kBlock;
    if (i < L.nout) L.z[1 + i] = out[u];
  }
}

template <bool HASY, bool IDENT, int U>
__global__ __launch_bounds__(kBlock) void k_band_one(const BandLaunch L) {
  band_qcomp_block<HASY, IDENT, U>(L, ptr_meta(L.op));
}

// Metadata of blocks that earlier steps of the same launch wrote: vector
// loads (never the scalar cache, which does not see those stores), at
// workgroup scope (the writers are lanes of this workgroup, ordered by the
// barrier between steps). The operands' exponents, which both qcomp passes
// resolve, are loaded once when the step starts (they do not change during
// the step: a block the step writes gets its exponent only at its end).
struct WgMeta {
  const int64_t* p[5];
  int64_t ex, ey;
  __device__ __forceinline__ int64_t operator()(int k, int f) const {
    if (f == kMetaExp && k == kOpX) return ex;
    if (f == kMetaExp && k == kOpY) return ey;
    return __hip_atomic_load(p[k] + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <bool HASY, bool IDENT>
__device__ __forceinline__ void band_step(const BandLaunch& L, int u) {
  const OpArgs& o = L.op;
  auto ld = [](const int64_t* q) {
    return __hip_atomic_load(q + kMetaExp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  const WgMeta m{{o.x_meta, o.y_meta, o.z_meta, o.g.a, o.g.b}, ld(o.x_meta), HASY ? ld(o.y_meta) : 0};
  if (u <= 1) band_qcomp_block<HASY, IDENT, 1>(L, m);
  else if (u <= 2) band_qcomp_block<HASY, IDENT, 2>(L, m);
  else if (u <= 4) band_qcomp_block<HASY, IDENT, 4>(L, m);
  else if (u <= 8) band_qcomp_block<HASY, IDENT, 8>(L, m);
  else band_qcomp_block<HASY, IDENT, 16>(L, m);
}

// A recorded sequence of finite-element steps in one workgroup: each step
// is one band op (both qcomp passes, as k_band_one) or the initialisation
// of a block (zero mantissas, metadata with exponent init_exp); a barrier
// separates consecutive steps, so a step reads what the previous ones
// wrote. The steps themselves are never written during the launch
// (__restrict__: their fields may come through the scalar cache).
__global__ __launch_bounds__(kBlock) void k_band_prog(const BandStep* __restrict__ steps, int nsteps) {
  for (int k = 0; k < nsteps; ++k) {
    const BandStep& S = steps[k];
    if (S.init_meta) {
      for (int64_t i = threadIdx.x; i < S.init_words; i += kBlock) S.init_mant[i] = 0;
      for (int i = threadIdx.x; i < kMetaSlots; i += kBlock) {
        int64_t v = 0;
        if (i >= kSetBase) {
          const int f = (i - kSetBase) % kSetStride;
          v = f == kAccMax ? INT64_MIN : (f == kAccMin ? INT64_MAX : 0);
        } else if (i < kMetaTicket) {
          v = i == kMetaExp ? S.init_exp : (i == kMetaMu ? 1 : 0);
        }
        S.init_meta[i] = v;
      }
    } else if (S.L.op.has_y) {
      if (S.L.taps) band_step<true, false>(S.L, S.u);
      else band_step<true, true>(S.L, S.u);
    } else {
      if (S.L.taps) band_step<false, false>(S.L, S.u);
      else band_step<false, true>(S.L, S.u);
    }
    __syncthreads();
  }
}

hipError_t launch_band_prog(const BandStep* steps, int nsteps, hipStream_t s) {
  hipLaunchKernelGGL(k_band_prog, dim3(1), dim3(kBlock), 0, s, steps, nsteps);
  return hipGetLastError();
}

template <bool HASY, bool IDENT>
static hipError_t band_one_go(const BandLaunch& L, hipStream_t s) {
  const dim3 g(1), b(kBlock);
  if (L.nout <= kBlock) hipLaunchKernelGGL((k_band_one<HASY, IDENT, 1>), g, b, 0, s, L);
  else if (L.nout <= 2 * kBlock) hipLaunchKernelGGL((k_band_one<HASY, IDENT, 2>), g, b, 0, s, L);
  else if (L.nout <= 4 * kBlock) hipLaunchKernelGGL((k_band_one<HASY, IDENT, 4>), g, b, 0, s, L);
  else if (L.nout <= 8 * kBlock) hipLaunchKernelGGL((k_band_one<HASY, IDENT, 8>), g, b, 0, s, L);
  else hipLaunchKernelGGL((k_band_one<HASY, IDENT, 16>), g, b, 0, s, L);
  return hipGetLastError();
}

template <int PASS, bool HASY, bool IDENT>
static hipError_t band_go(const BandLaunch& L, hipStream_t s) {
  const int64_t blocks = (L.nout + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_band<PASS, HASY, IDENT>),
                     dim3((unsigned)(blocks < kMaxBlocks ? (blocks > 0 ? blocks : 1) : kMaxBlocks)),
                     dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

hipError_t launch_band(const BandLaunch& L, hipStream_t s) {
  const bool q1 = L.op.mode == kModeQ1;
  const bool id = L.taps == nullptr;
  if (L.op.has_y) {
    if (id) return q1 ? band_go<kQ1, true, true>(L, s) : band_go<kOut, true, true>(L, s);
    return q1 ? band_go<kQ1, true, false>(L, s) : band_go<kOut, true, false>(L, s);
  }
  if (id) return q1 ? band_go<kQ1, false, true>(L, s) : band_go<kOut, false, true>(L, s);
  return q1 ? band_go<kQ1, false, false>(L, s) : band_go<kOut, false, false>(L, s);
}

hipError_t launch_band_qcomp1(const BandLaunch& L, hipStream_t s) {
  if (L.nout > kBandOneMax) return hipErrorInvalidValue;
  const bool id = L.taps == nullptr;
  if (L.op.has_y) return id ? band_one_go<true, true>(L, s) : band_one_go<true, false>(L, s);
  return id ? band_one_go<false, true>(L, s) : band_one_go<false, false>(L, s);
}

}  // namespace bfpk
