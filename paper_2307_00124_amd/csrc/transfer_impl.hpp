// Grid transfers with full 3^d taps, fused with the exact epilogue:
//   restriction   z[I] = Q(alpha * sum_o t[o] x[2I + o] + beta * y[I])   (qspmv R)
//   prolongation  z[p] = Q(alpha * sum_o t[o] u[p + o] + beta * y[p])    (qspmv P /
//                 qgemv(P, d, y, -1, 1) of the V-cycle), u = x on the even
//                 fine nodes, zero elsewhere.
// A prolongation thread owns one coarse cell C and writes the 2^d fine nodes
// 2C + delta (delta in {0,1}^d): a fine node takes tap o = 2J - p from each
// coarse corner J = C + eps with eps_k = 0 where delta_k = 0.
#pragma once

#include "epilogue.hpp"

#include <utility>

namespace bfpk {

template <int ND>
__device__ __forceinline__ int tap_index(const int (&o)[3]) {
  return ND == 2 ? (o[1] + 1) * 3 + (o[2] + 1) : ((o[0] + 1) * 3 + (o[1] + 1)) * 3 + (o[2] + 1);
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): a loop
// whose index is a compile-time constant from the start
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>());
}

// one coarse output point per thread; work items: (output row, run of 256 points) pairs, grid-strided over at
// most kMaxBlocks blocks
template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_restrict(const TransferLaunch L) {
  const int64_t nc = L.n_out;
  const int64_t sf = L.n_in + 2, sc = nc + 2;
  const int64_t nchunk = (nc + kBlock - 1) / kBlock;
  const int64_t items = (ND == 3 ? nc * nc : nc) * nchunk;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  Epi<PASS, HASY> E;
  E.init(L.op);
  with_fast(E, [&](auto fast_tag) {
  constexpr int VAR = decltype(fast_tag)::value;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t row = it / nchunk;                       // 0 .. nc^(ND-1) - 1
    const int64_t xc = (it % nchunk) * kBlock + threadIdx.x + 1;
    int64_t zc = 0, yc;
    if (ND == 3) { zc = row / nc + 1; yc = row % nc + 1; } else { yc = row + 1; }
    if (xc > nc) continue;
    // all 3^ND loads of the point are issued together (compile-time offsets
    // and taps), not one fine row after the other
    int64_t g = 0;
    static_for<ND == 3 ? 3 : 1>([&](auto iz_) {
      constexpr int oz = ND == 3 ? decltype(iz_)::value - 1 : 0;
      static_for<3>([&](auto iy_) {
        constexpr int oy = decltype(iy_)::value - 1;
        const int64_t frow = ND == 3 ? (2 * zc + oz) * sf + (2 * yc + oy) : (2 * yc + oy);
        const TX* xr = X + frow * L.px + 2 * xc;
        static_for<3>([&](auto ix_) {
          constexpr int ox = decltype(ix_)::value - 1;
          constexpr int ti = ND == 2 ? (oy + 1) * 3 + (ox + 1) : ((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1);
          g += (int64_t)L.taps[ti] * (int64_t)xr[ox];
        });
      });
    });
    const int64_t crow = ND == 3 ? zc * sc + yc : yc;
    const int64_t yv = HASY ? (int64_t)Y[crow * L.py + xc] : 0;
    const int64_t v = E.template put<VAR>(g, yv, true);
    if (PASS != kQ1) Z[crow * L.pz + xc] = (TZ)v;
  }
  });
  E.finish();
}

template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_prolong(const TransferLaunch L) {
  const int64_t nc = L.n_in, nf = L.n_out;
  const int64_t sf = nf + 2, sc = nc + 2;
  const int64_t cells = nc + 1;                               // coarse cells per dim
  const int64_t nchunk = (cells + kBlock - 1) / kBlock;
  const int64_t items = (ND == 3 ? cells * cells : cells) * nchunk;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  Epi<PASS, HASY> E;
  E.init(L.op);
  with_fast(E, [&](auto fast_tag) {
  constexpr int VAR = decltype(fast_tag)::value;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t row = it / nchunk;
    const int64_t cx = (it % nchunk) * kBlock + threadIdx.x;
    int64_t cz = 0, cy;
    if (ND == 3) { cz = row / cells; cy = row % cells; } else { cy = row; }
    if (cx >= cells) continue;
    int64_t cv[2][2][2];
#pragma unroll
    for (int ez = 0; ez < (ND == 3 ? 2 : 1); ++ez)
#pragma unroll
      for (int ey = 0; ey < 2; ++ey) {
        const int64_t crow = ND == 3 ? (cz + ez) * sc + (cy + ey) : (cy + ey);
        cv[ez][ey][0] = X[crow * L.px + cx];
        cv[ez][ey][1] = X[crow * L.px + cx + 1];
      }
#pragma unroll
    for (int dz = 0; dz < (ND == 3 ? 2 : 1); ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        const int64_t fz = 2 * cz + dz, fy = 2 * cy + dy;
        const bool row_in = (ND == 2 || (fz >= 1 && fz <= nf)) && fy >= 1 && fy <= nf;
        const int64_t frow = ND == 3 ? fz * sf + fy : fy;
        int64_t outv[2] = {0, 0};
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int64_t fx = 2 * cx + dx;
          if (!row_in || fx < 1 || fx > nf) continue;
          int64_t g = 0;
          int o[3];
#pragma unroll
          for (int ez = 0; ez < 2; ++ez) {
            if (ND == 2 && ez) continue;
            if (ND == 3 && !dz && ez) continue;
#pragma unroll
            for (int ey = 0; ey < 2; ++ey) {
              if (!dy && ey) continue;
#pragma unroll
              for (int ex = 0; ex < 2; ++ex) {
                if (!dx && ex) continue;
                o[0] = ND == 3 ? (dz ? 2 * ez - 1 : 0) : 0;
                o[1] = dy ? 2 * ey - 1 : 0;
                o[2] = dx ? 2 * ex - 1 : 0;
                g += (int64_t)L.taps[tap_index<ND>(o)] * cv[ez][ey][ex];
              }
            }
          }
          const int64_t yv = HASY ? (int64_t)Y[frow * L.py + fx] : 0;
          outv[dx] = E.template put<VAR>(g, yv, true);
          if (PASS != kQ1) Z[frow * L.pz + fx] = (TZ)outv[dx];
        }
      }
  }
  });
  E.finish();
}

template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
static hipError_t transfer_go(const TransferLaunch& L, hipStream_t s) {
  if (L.kind == 1) {
    const int64_t nc = L.n_out;
    const int64_t rows = ND == 3 ? nc * nc : nc;
    const int64_t items = rows * ((nc + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_restrict<ND, TX, TY, TZ, PASS, HASY>),
                       dim3((unsigned)(items < kMaxBlocks ? items : kMaxBlocks)), dim3(kBlock), 0,
                       s, L);
  } else {
    const int64_t cells = L.n_in + 1;
    const int64_t rows = ND == 3 ? cells * cells : cells;
    const int64_t items = rows * ((cells + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_prolong<ND, TX, TY, TZ, PASS, HASY>),
                       dim3((unsigned)(items < kMaxBlocks ? items : kMaxBlocks)), dim3(kBlock), 0,
                       s, L);
  }
  return hipGetLastError();
}

template <int ND>
hipError_t transfer_nd(const TransferLaunch& L, hipStream_t s) {
  const bool q1 = L.op.mode == kModeQ1;
  return with_type(L.xbits, [&](auto tx) {
    using TX = decltype(tx);
    if (!L.op.has_y) {
      if (q1) return transfer_go<ND, TX, int32_t, int32_t, kQ1, false>(L, s);
      return with_type(L.zbits, [&](auto tz) {
        return transfer_go<ND, TX, int32_t, decltype(tz), kOut, false>(L, s);
      });
    }
    return with_type(L.ybits, [&](auto ty) {
      using TY = decltype(ty);
      if (q1) return transfer_go<ND, TX, TY, int32_t, kQ1, true>(L, s);
      return with_type(L.zbits, [&](auto tz) {
        return transfer_go<ND, TX, TY, decltype(tz), kOut, true>(L, s);
      });
    });
  });
}

}  // namespace bfpk
