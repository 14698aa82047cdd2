// Star stencils (centre + 2 ndim face taps) on one grid: the 5-point (2D)
// and 7-point (3D) operators A' of the D = I setup, fused with the exact
// alpha A x + beta y epilogue (the exact gemv rows of Appendix B) and the
// qcomp / nnqcomp quantization.
//
// Layout: each wave owns 256 consecutive x columns (4 per lane, one 16-byte
// load for int32 mantissas) and marches through `rows` rows (2D, in y) or
// planes (3D, in z), keeping the previous / current / next line in
// registers, so each input line is read from HBM once per march. The x
// neighbours come from adjacent lanes (wave shuffles); only the two wave-edge
// lanes load a single extra element. In 3D the y neighbours are the lines
// of the waves above / below, read through L2.
//
// 2D blocks: the 4 waves of a block take WX adjacent column segments times
// 4 / WX row bands (WX = 4 on wide grids), and tiles are assigned in an
// XCD-aware order. Consecutive dispatch ids land on different XCDs (each
// with its own L2), so tile = xcd_tile(id) gives every XCD a contiguous run
// of tiles: the wave-edge columns and the halo rows a tile shares with its
// neighbours are then fetched from HBM once and re-read from the same L2.
#pragma once

#include "epilogue.hpp"

namespace bfpk {

// U rows per batch, software-pipelined: the loads of batch i+1 (U new x
// lines, U y lines, the wave-edge neighbours) are issued before batch i is
// computed and stored. Stores count in the same vector-memory counter as
// loads, so issuing the next loads first keeps the wait for them from also
// waiting on this batch's store acknowledgements.
template <typename TX, typename TY, int U, bool HASY, bool YX>
__device__ __forceinline__ void star2d_fetch(const TX* X, const TY* Y, int64_t r, int64_t n,
                                             int64_t px, int64_t py, int64_t c, int lane,
                                             bool act, bool act_y, int32_t (&xl)[U][4],
                                             int32_t (&yl)[U][4], int32_t (&eg)[U]) {
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int64_t rr = r + 1 + k;                    // x lines r+1 .. r+U
    ld4(X, rr * px + c, xl[k], act && rr <= n + 1);
    if (HASY && !YX) ld4(Y, (r + k) * py + c, yl[k], act_y && r + k <= n);
    else yl[k][0] = yl[k][1] = yl[k][2] = yl[k][3] = 0;
    // lane 0 needs column c-1, lane 63 column c+4 (other lanes read a
    // harmless in-range value and ignore it)
    const int64_t re = r + k <= n ? r + k : n;
    const int64_t ce = lane == 0 ? c - 1 : c + 4;
    eg[k] = ld1(X, re * px + ce, (lane == 0 || lane == 63) && ce >= 0 && ce < px);
  }
}

constexpr int kXcds = 8;

// dispatch id -> tile, a bijection on [0, nblk) under which XCD k (the
// dispatch ids congruent to k mod 8) receives the contiguous tiles
// [k q + min(k, r), ...) with q = nblk / 8, r = nblk % 8
__device__ __forceinline__ int64_t xcd_tile(int64_t id, int64_t nblk) {
  const int64_t q = nblk / kXcds, r = nblk % kXcds;
  const int64_t k = id % kXcds, j = id / kXcds;
  return k * q + (k < r ? k : r) + j;
}

// YX: y is x itself (the relaxation): its entries are the centre values
template <typename TX, typename TY, typename TZ, int PASS, bool HASY, bool WIDE, int U, bool YX>
__global__ __launch_bounds__(kBlock) void k_star2d(const StarLaunch L) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t n = L.n, px = L.px, py = L.py, pz = L.pz;
  const int wx = wv % L.wx, wy = wv / L.wx;
  const int64_t tiles_x = gridDim.x;
  const int64_t tile = xcd_tile(blockIdx.x + (int64_t)blockIdx.y * gridDim.x,
                                (int64_t)gridDim.x * gridDim.y);
  const int64_t c = ((tile % tiles_x) * L.wx + wx) * 256 + lane * 4;
  const bool act = c < px, act_y = c < py, act_z = c < pz;
  const int64_t r0 = 1 + ((tile / tiles_x) * (4 / L.wx) + wy) * L.rows;
  int64_t r1 = r0 + L.rows;
  if (r1 > n + 1) r1 = n + 1;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  const int32_t t0 = L.taps[0], txm = L.taps[1], txp = L.taps[2], tym = L.taps[3],
                typ = L.taps[4];
  // the first batch's loads are issued before the epilogue reads the
  // operands' metadata (they do not depend on it), so the two round trips
  // overlap
  const bool live = r0 < r1;
  int32_t win[U + 2][4];                   // lines r-1 .. r+U of the current batch
  int32_t yv[U][4], eg[U];
  ld4(X, (r0 - 1) * px + c, win[0], act && live);
  ld4(X, r0 * px + c, win[1], act && live);
  star2d_fetch<TX, TY, U, HASY, YX>(X, Y, r0, n, px, py, c, lane, act && live, act_y && live,
                                    *reinterpret_cast<int32_t(*)[U][4]>(&win[2]), yv, eg);
  Epi<PASS, HASY> E;
  E.init(L.op);
  bool colok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colok[q] = c + q >= 1 && c + q <= n;
  if (live) with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    int32_t nx[U][4], ny[U][4], ne[U];     // the next batch in flight
    for (int64_t r = r0; r < r1; r += U) {
      star2d_fetch<TX, TY, U, HASY, YX>(X, Y, r + U, n, px, py, c, lane, act, act_y, nx, ny, ne);
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int32_t* up = win[k];
        const int32_t* cur = win[k + 1];
        const int32_t* dn = win[k + 2];
        int32_t left = __shfl_up(cur[3], 1, 64);
        int32_t right = __shfl_down(cur[0], 1, 64);
        if (lane == 0) left = eg[k];
        if (lane == 63) right = eg[k];
        const bool row_ok = r + k < r1;
        int64_t out[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t xl = q ? cur[q - 1] : left;
          const int32_t xr = q < 3 ? cur[q + 1] : right;
          int64_t g;
          if (WIDE)
            g = (int64_t)t0 * cur[q] + (int64_t)txm * xl + (int64_t)txp * xr +
                (int64_t)tym * up[q] + (int64_t)typ * dn[q];
          else
            g = (int64_t)(t0 * cur[q] + txm * xl + txp * xr + tym * up[q] + typ * dn[q]);
          out[q] = E.template put<VAR>(g, YX ? cur[q] : yv[k][q], row_ok && colok[q]);
        }
        if (PASS != kQ1 && act_z && row_ok) st4(Z, (r + k) * pz + c, out);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        win[0][q] = win[U][q];
        win[1][q] = win[U + 1][q];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        eg[k] = ne[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          win[k + 2][q] = nx[k][q];
          yv[k][q] = ny[k][q];
        }
      }
    }
  });
  E.finish();
}

// 3D: each wave owns a stack of 4 consecutive y rows of one 256-column
// segment and marches through `rows` z planes. It keeps plane z-1 (4 rows),
// plane z (the 4 rows and the halo rows above and below) and plane z+1 in
// registers, so y and z neighbours come from registers and only the two
// halo rows are extra loads; the loads of plane z+2 (and of the next
// plane's halo, y and edge values) are issued before plane z is computed.
// A block's 4 waves take 4 consecutive stacks (16 rows), so their halo rows
// are lines the neighbouring waves load anyway.
constexpr int kYS = 4;

template <typename TX, typename TY>
__device__ __forceinline__ void star3d_plane(const TX* X, const TY* Y, int64_t z, int64_t y0,
                                             int64_t n, int64_t side, int64_t px, int64_t py,
                                             int64_t c, int lane, bool act, bool act_y,
                                             bool hasy, int32_t (&hm)[4], int32_t (&hp)[4],
                                             int32_t (&yv)[kYS][4], int32_t (&eg)[kYS]) {
  // plane z: halo rows y0 - 1 and y0 + kYS, y operand and edge values of
  // rows y0 .. y0 + kYS - 1
  const bool zok = z <= n + 1;
  ld4(X, (z * side + y0 - 1) * px + c, hm, act && zok);
  ld4(X, (z * side + y0 + kYS) * px + c, hp, act && zok && y0 + kYS <= n + 1);
  const int64_t ce = lane == 0 ? c - 1 : c + 4;
  const bool eok = (lane == 0 || lane == 63) && ce >= 0 && ce < px;
#pragma unroll
  for (int k = 0; k < kYS; ++k) {
    const int64_t y = y0 + k;
    const bool rok = zok && y <= n + 1;
    if (hasy) ld4_nt(Y, (z * side + y) * py + c, yv[k], act_y && rok && z <= n && y <= n);
    eg[k] = ld1(X, (z * side + y) * px + ce, eok && rok);
  }
}

template <typename TX>
__device__ __forceinline__ void star3d_rows4(const TX* X, int64_t z, int64_t y0, int64_t n,
                                             int64_t side, int64_t px, int64_t c, bool act,
                                             int32_t (&v)[kYS][4]) {
#pragma unroll
  for (int k = 0; k < kYS; ++k)
    ld4(X, (z * side + y0 + k) * px + c, v[k], act && z <= n + 1 && y0 + k <= n + 1);
}

template <typename TX, typename TY, typename TZ, int PASS, bool HASY, bool YX>
__global__ __launch_bounds__(kBlock) void k_star3d(const StarLaunch L) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t n = L.n, px = L.px, py = L.py, pz = L.pz;
  const int64_t side = n + 2;
  // XCD-aware tile order (see xcd_tile): y- and z-neighbouring tiles, which
  // share halo lines, mostly run on the same XCD
  const int64_t gx = gridDim.x, gy = gridDim.y;
  const int64_t tile = xcd_tile(blockIdx.x + gx * (blockIdx.y + gy * (int64_t)blockIdx.z),
                                gx * gy * gridDim.z);
  const int64_t bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
  const int64_t c = bx * 256 + lane * 4;
  const bool act = c < px, act_y = c < py, act_z = c < pz;
  const int64_t y0 = 1 + (by * 4 + wv) * kYS;
  const int64_t z0 = 1 + bz * L.rows;
  int64_t z1 = z0 + L.rows;
  if (z1 > n + 1) z1 = n + 1;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  const int32_t t0 = L.taps[0], txm = L.taps[1], txp = L.taps[2], tym = L.taps[3],
                typ = L.taps[4], tzm = L.taps[5], tzp = L.taps[6];
  bool colok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colok[q] = c + q >= 1 && c + q <= n;
  Epi<PASS, HASY> E;
  E.init(L.op);
  if (y0 <= n && z0 < z1) with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    int32_t pa[kYS][4], pb[kYS][4], pc[kYS][4];   // planes z-1, z, z+1 (rows y0..)
    int32_t hm[4], hp[4], yv[kYS][4], eg[kYS];     // plane z: halo rows, y, edges
    int32_t nc[kYS][4], nhm[4], nhp[4], nyv[kYS][4], neg[kYS];   // next plane in flight
    star3d_rows4(X, z0 - 1, y0, n, side, px, c, act, pa);
    star3d_rows4(X, z0, y0, n, side, px, c, act, pb);
    star3d_rows4(X, z0 + 1, y0, n, side, px, c, act, pc);
    star3d_plane(X, Y, z0, y0, n, side, px, py, c, lane, act, act_y, HASY && !YX, hm, hp, yv, eg);
    for (int64_t z = z0; z < z1; ++z) {
      star3d_rows4(X, z + 2, y0, n, side, px, c, act, nc);
      star3d_plane(X, Y, z + 1, y0, n, side, px, py, c, lane, act, act_y, HASY && !YX, nhm, nhp,
                   nyv, neg);
#pragma unroll
      for (int k = 0; k < kYS; ++k) {
        const int32_t* cur = pb[k];
        const int32_t* up = k ? pb[k - 1] : hm;
        const int32_t* dn = k < kYS - 1 ? pb[k + 1] : hp;
        int32_t left = __shfl_up(cur[3], 1, 64);
        int32_t right = __shfl_down(cur[0], 1, 64);
        if (lane == 0) left = eg[k];
        if (lane == 63) right = eg[k];
        const bool row_ok = y0 + k <= n;
        int64_t out[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t xl = q ? cur[q - 1] : left;
          const int32_t xr = q < 3 ? cur[q + 1] : right;
          const int64_t g = (int64_t)t0 * cur[q] + (int64_t)txm * xl + (int64_t)txp * xr +
                            (int64_t)tym * up[q] + (int64_t)typ * dn[q] +
                            (int64_t)tzm * pa[k][q] + (int64_t)tzp * pc[k][q];
          out[q] = E.template put<VAR>(g, YX ? cur[q] : yv[k][q], row_ok && colok[q]);
        }
        if (PASS != kQ1 && act_z && row_ok) st4_nt(Z, (z * side + y0 + k) * pz + c, out);
      }
#pragma unroll
      for (int k = 0; k < kYS; ++k) {
        eg[k] = neg[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          pa[k][q] = pb[k][q];
          pb[k][q] = pc[k][q];
          pc[k][q] = nc[k][q];
          yv[k][q] = nyv[k][q];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hm[q] = nhm[q];
        hp[q] = nhp[q];
      }
    }
  });
  E.finish();
}

// ----------------------------------------------------------- launchers --

template <typename TX, typename TY, typename TZ, int PASS, bool HASY, bool YX = false>
static hipError_t star_go(const StarLaunch& L0, hipStream_t s) {
  StarLaunch L = L0;
  const int64_t n = L.n;
  const int rows = L.rows > 0 ? L.rows : 1;
  if (L.ndim == 2) {
    const int64_t segs = (n + 1 + 255) / 256, bands = (n + rows - 1) / rows;
    const int wx = L.wx;
    dim3 grid((unsigned)((segs + wx - 1) / wx), (unsigned)((bands + 4 / wx - 1) / (4 / wx)));
    if ((int64_t)grid.x * grid.y > kMaxSlotBlocks) L.op.slots = nullptr;
    if (rows >= 4 && rows % 4 == 0) {
      if (L.wide)
        hipLaunchKernelGGL((k_star2d<TX, TY, TZ, PASS, HASY, true, 4, YX>), grid, dim3(kBlock), 0, s, L);
      else
        hipLaunchKernelGGL((k_star2d<TX, TY, TZ, PASS, HASY, false, 4, YX>), grid, dim3(kBlock), 0, s, L);
    } else {
      if (L.wide)
        hipLaunchKernelGGL((k_star2d<TX, TY, TZ, PASS, HASY, true, 1, YX>), grid, dim3(kBlock), 0, s, L);
      else
        hipLaunchKernelGGL((k_star2d<TX, TY, TZ, PASS, HASY, false, 1, YX>), grid, dim3(kBlock), 0, s, L);
    }
  } else {
    dim3 grid((unsigned)((n + 1 + 255) / 256), (unsigned)((n + 4 * kYS - 1) / (4 * kYS)),
              (unsigned)((n + rows - 1) / rows));
    if ((int64_t)grid.x * grid.y * grid.z > kMaxSlotBlocks) L.op.slots = nullptr;
    hipLaunchKernelGGL((k_star3d<TX, TY, TZ, PASS, HASY, YX>), grid, dim3(kBlock), 0, s, L);
  }
  return hipGetLastError();
}

// launch_star for one storage type of x
template <typename TX>
hipError_t star_for_x(const StarLaunch& L, hipStream_t s) {
  const bool q1 = L.op.mode == kModeQ1;
  if (!L.op.has_y) {
    if (q1) return star_go<TX, int32_t, int32_t, kQ1, false>(L, s);
    return with_type(L.zbits, [&](auto tz) {
      return star_go<TX, int32_t, decltype(tz), kOut, false>(L, s);
    });
  }
  if (L.y_is_x) {   // the relaxation: y is x, read once
    if (q1) return star_go<TX, TX, int32_t, kQ1, true, true>(L, s);
    return with_type(L.zbits, [&](auto tz) {
      return star_go<TX, TX, decltype(tz), kOut, true, true>(L, s);
    });
  }
  return with_type(L.ybits, [&](auto ty) {
    using TY = decltype(ty);
    if (q1) return star_go<TX, TY, int32_t, kQ1, true>(L, s);
    return with_type(L.zbits, [&](auto tz) {
      return star_go<TX, TY, decltype(tz), kOut, true>(L, s);
    });
  });
}

}  // namespace bfpk
