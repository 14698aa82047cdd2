// Grid transfers with full 3^d taps, fused with the exact epilogue:
//   restriction   z[I] = Q(alpha * sum_o t[o] x[2I + o] + beta * y[I])   (qspmv R)
//   prolongation  z[p] = Q(alpha * sum_(J: |2J-p| <= 1) t[2J - p] x[J] + beta * y[p])
//                 (qspmv P, and the V-cycle's qgemv(P, d, y, -1, 1))
//
// Both are streaming kernels laid out like the star kernels: a wave owns a
// segment of 256 output columns (4 per lane, one 16-byte store per output
// line) and marches through a band of coarse rows (2D) or coarse planes
// (3D), so every input line is loaded once per march with wide contiguous
// loads and every output line is stored once.
//
//  * Prolongation: lane columns c..c+3 (c a multiple of 4) of a fine line
//    take the coarse values at c/2, c/2 + 1 (one 2-element load) and c/2 + 2
//    (the next lane's first value, by a wave shuffle). Even fine lines come
//    from one coarse line (offset 0), odd ones from the two around them
//    (offsets -1 and +1); in 3D the same holds for planes. A 2D wave marches
//    over coarse rows J, writing fine rows 2J and 2J + 1; a 3D wave owns one
//    coarse row J_y (fine rows 2J_y, 2J_y + 1) and marches over coarse
//    planes J_z, writing fine planes 2J_z and 2J_z + 1.
//  * Restriction: lane columns C..C+3 of a coarse line read the fine values
//    2C - 1 .. 2C + 7 (an aligned 8-element load and the previous lane's
//    last value by a shuffle). Coarse line I sums fine lines 2I - 1, 2I,
//    2I + 1; the march loads fine lines 2I and 2I + 1 per step and carries
//    the share of fine line 2I + 1 in coarse line I + 1 (offset -1) to the
//    next step, so no fine line is read twice by a wave.
//
// Tiles (one per block: 4 waves on 4 consecutive bands of one segment) are
// assigned in the XCD-aware order of the star kernels.
#pragma once

#include "epilogue.hpp"

namespace bfpk {

constexpr int kTrXcds = 8;

__device__ __forceinline__ int64_t tr_xcd_tile(int64_t id, int64_t nblk) {
  const int64_t q = nblk / kTrXcds, r = nblk % kTrXcds;
  const int64_t k = id % kTrXcds, j = id / kTrXcds;
  return k * q + (k < r ? k : r) + j;
}

// NV consecutive mantissas from an index aligned to NV (branch-free: an
// out-of-range request reads element 0 and yields zeros)
template <typename T, int NV>
__device__ __forceinline__ void ldv(const T* base, int64_t off, int32_t (&v)[NV], bool ok) {
  struct alignas(NV * sizeof(T)) V {
    T v[NV];
  };
  const V q = *reinterpret_cast<const V*>(base + (ok ? off : 0));
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = ok ? (int32_t)q.v[k] : 0;
}

// ------------------------------------------------------- prolongation ---

// One coarse line's share in 4 fine columns: tap row T (offsets -1, 0, +1
// in x) applied to the coarse values a[0..2] at c/2 .. c/2 + 2.
__device__ __forceinline__ void pro_line(const int32_t* T, const int32_t (&a)[3], int64_t (&g)[4]) {
  g[0] += (int64_t)T[1] * a[0];
  g[1] += (int64_t)T[0] * a[0] + (int64_t)T[2] * a[1];
  g[2] += (int64_t)T[1] * a[1];
  g[3] += (int64_t)T[0] * a[1] + (int64_t)T[2] * a[2];
}

// coarse values c/2, c/2 + 1 of one coarse line (and c/2 + 2 from the next lane)
template <typename TX>
__device__ __forceinline__ void pro_load(const TX* X, int64_t row_off, int64_t cc, int64_t pc,
                                         bool rok, int lane, int32_t (&a)[3]) {
  int32_t p[2];
  ldv<TX, 2>(X, row_off + cc, p, rok && cc < pc);
  // lane 63 needs c/2 + 2 of its own; the others take it from the next lane
  const int32_t e = ld1(X, row_off + cc + 2, rok && lane == 63 && cc + 2 < pc);
  a[0] = p[0];
  a[1] = p[1];
  a[2] = p[0];   // replaced below by the shuffle / edge value
  const int32_t nb = __shfl_down(p[0], 1, 64);
  a[2] = lane == 63 ? e : nb;
}

template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_prolong(const TransferLaunch L) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nc = L.n_in, nf = L.n_out;
  const int64_t sc = nc + 2, sf = nf + 2;
  const int64_t px = L.px, py = L.py, pz = L.pz;
  const int64_t segs = gridDim.x;
  const int64_t tile = tr_xcd_tile(blockIdx.x + (int64_t)gridDim.x * blockIdx.y,
                                   (int64_t)gridDim.x * gridDim.y);
  const int64_t c = (tile % segs) * 256 + lane * 4;       // fine columns c..c+3
  const int64_t cc = c / 2;                                // coarse columns cc..cc+2
  const int64_t band = (tile / segs) * 4 + wv;
  // 2D: band of coarse rows; 3D: (coarse row, band of coarse planes)
  const int64_t nbz = (nc + 1 + L.rows - 1) / L.rows;     // bands per coarse row (3D)
  const int64_t jy3 = ND == 3 ? band / nbz : 0;
  const int64_t b0 = (ND == 3 ? band % nbz : band) * L.rows;   // first coarse row / plane
  int64_t b1 = b0 + L.rows;
  if (b1 > nc + 1) b1 = nc + 1;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  bool colok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colok[q] = c + q >= 1 && c + q <= nf;
  const bool act_y = c < py, act_z = c < pz;
  const bool live = b0 < b1 && (ND == 2 || jy3 <= nc);
  // 2D: the first two coarse lines (and y rows) are loaded before the
  // epilogue reads the operands' metadata, so the two round trips overlap
  int32_t A2[3], B2[3], y0[4], y1[4];
  if (ND == 2) {
    pro_load(X, b0 * px, cc, px, live, lane, A2);
    pro_load(X, (b0 + 1) * px, cc, px, live && b0 + 1 <= nc + 1, lane, B2);
    if (HASY) {
      ld4(Y, (2 * b0) * py + c, y0, live && act_y && 2 * b0 <= nf);
      ld4(Y, (2 * b0 + 1) * py + c, y1, live && act_y && 2 * b0 + 1 <= nf);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) y0[q] = y1[q] = 0;
    }
  }
  Epi<PASS, HASY> E;
  E.init(L.op);
  if (live) with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    // fine line (plane fz, row fy) from the coarse lines held in A (line
    // index b) and B (line b + 1); 2D: A, B are coarse rows b, b + 1
    // 3D: A[r], B[r] are rows jy3 + r of coarse planes b, b + 1
    auto emit = [&](int64_t fz, int64_t fy, const int64_t (&g)[4], const int32_t (&yv)[4]) {
      const bool line_ok = fy >= 1 && fy <= nf && (ND == 2 || (fz >= 1 && fz <= nf));
      int64_t out[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = E.template put<VAR>(g[q], yv[q], line_ok && colok[q]);
      if (PASS != kQ1 && act_z && line_ok)
        st4(Z, ((ND == 3 ? fz * sf : 0) + fy) * pz + c, out);
    };
    if (ND == 2) {
      const int32_t* T0 = &t[0];   // offset -1 in y
      const int32_t* T1 = &t[3];   // offset 0
      const int32_t* T2 = &t[6];   // offset +1
      int32_t A[3], B[3], Cn[3], y0n[4], y1n[4];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        A[q] = A2[q];
        B[q] = B2[q];
      }
      for (int64_t J = b0; J < b1; ++J) {
        // loads of the next step first
        pro_load(X, (J + 2) * px, cc, px, J + 2 <= nc + 1, lane, Cn);
        if (HASY) {
          ld4(Y, (2 * J + 2) * py + c, y0n, act_y && 2 * J + 2 <= nf);
          ld4(Y, (2 * J + 3) * py + c, y1n, act_y && 2 * J + 3 <= nf);
        }
        int64_t ge[4] = {0, 0, 0, 0}, go[4] = {0, 0, 0, 0};
        pro_line(T1, A, ge);                  // fine row 2J: coarse row J
        pro_line(T0, A, go);                  // fine row 2J + 1: rows J (-1) and J + 1 (+1)
        pro_line(T2, B, go);
        emit(0, 2 * J, ge, y0);
        emit(0, 2 * J + 1, go, y1);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          A[q] = B[q];
          B[q] = Cn[q];
        }
        if (HASY) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            y0[q] = y0n[q];
            y1[q] = y1n[q];
          }
        }
      }
    } else {
      // taps t[((oz + 1) * 3 + (oy + 1)) * 3 + ox + 1]
      int32_t A[2][3], B[2][3], Cn[2][3];
      int32_t yv[2][2][4], yn[2][2][4];     // [fine plane parity][fine row parity]
      auto load_plane = [&](int64_t jz, int32_t (&P)[2][3]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
          pro_load(X, (jz * sc + jy3 + r) * px, cc, px, jz <= nc + 1 && jy3 + r <= nc + 1, lane,
                   P[r]);
      };
      auto load_y = [&](int64_t jz, int32_t (&V)[2][2][4]) {
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            const int64_t fz = 2 * jz + dz, fy = 2 * jy3 + dy;
            if (HASY) ld4(Y, (fz * sf + fy) * py + c, V[dz][dy], act_y && fz <= nf && fy <= nf);
            else V[dz][dy][0] = V[dz][dy][1] = V[dz][dy][2] = V[dz][dy][3] = 0;
          }
      };
      load_plane(b0, A);
      load_plane(b0 + 1, B);
      load_y(b0, yv);
      for (int64_t J = b0; J < b1; ++J) {
        load_plane(J + 2, Cn);
        if (HASY) load_y(J + 1, yn);
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            int64_t g[4] = {0, 0, 0, 0};
            // fine plane 2J + dz, fine row 2 jy3 + dy: coarse planes J (offset
            // -dz) and J + 1 (offset +1, odd planes only), rows likewise
#pragma unroll
            for (int ez = 0; ez < 2; ++ez) {
              if (!dz && ez) continue;
              const int oz = dz ? 2 * ez - 1 : 0;
#pragma unroll
              for (int ey = 0; ey < 2; ++ey) {
                if (!dy && ey) continue;
                const int oy = dy ? 2 * ey - 1 : 0;
                const int32_t* T = &t[((oz + 1) * 3 + (oy + 1)) * 3];
                pro_line(T, ez ? B[ey] : A[ey], g);
              }
            }
            emit(2 * J + dz, 2 * jy3 + dy, g, yv[dz][dy]);
          }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            A[r][q] = B[r][q];
            B[r][q] = Cn[r][q];
          }
        if (HASY) {
#pragma unroll
          for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
              for (int q = 0; q < 4; ++q) yv[dz][dy][q] = yn[dz][dy][q];
        }
      }
    }
  });
  E.finish();
}

// -------------------------------------------------------- restriction ---

// fine values 2C - 1 .. 2C + 7 of one fine line (w[0] = 2C - 1)
template <typename TX>
__device__ __forceinline__ void res_load(const TX* X, int64_t row_off, int64_t C, int64_t pf,
                                         bool rok, int lane, int32_t (&w)[9]) {
  int32_t v[8];
  ldv<TX, 8>(X, row_off + 2 * C, v, rok && 2 * C < pf);
  const int32_t e = ld1(X, row_off + 2 * C - 1, rok && lane == 0 && C >= 1 && 2 * C - 1 < pf);
  const int32_t prev = __shfl_up(v[7], 1, 64);
  w[0] = lane == 0 ? e : prev;
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k + 1] = v[k];
}

// one fine line's share in 4 coarse columns, tap row T (x offsets -1, 0, +1)
__device__ __forceinline__ void res_line(const int32_t* T, const int32_t (&w)[9], int64_t (&g)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    g[k] += (int64_t)T[0] * w[2 * k] + (int64_t)T[1] * w[2 * k + 1] + (int64_t)T[2] * w[2 * k + 2];
}

template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
__global__ __launch_bounds__(kBlock) void k_restrict(const TransferLaunch L) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nc = L.n_out, nf = L.n_in;
  const int64_t sc = nc + 2, sf = nf + 2;
  const int64_t px = L.px, py = L.py, pz = L.pz;
  const int64_t segs = gridDim.x;
  const int64_t tile = tr_xcd_tile(blockIdx.x + (int64_t)gridDim.x * blockIdx.y,
                                   (int64_t)gridDim.x * gridDim.y);
  const int64_t C = (tile % segs) * 256 + lane * 4;       // coarse columns C..C+3
  const int64_t band = (tile / segs) * 4 + wv;
  const int64_t nb = (nc + L.rows - 1) / L.rows;          // bands per coarse row (3D)
  const int64_t yc3 = ND == 3 ? band / nb + 1 : 0;
  const int64_t b0 = (ND == 3 ? band % nb : band) * L.rows + 1;   // first coarse row / plane
  int64_t b1 = b0 + L.rows;
  if (b1 > nc + 1) b1 = nc + 1;
  const TX* X = static_cast<const TX*>(L.x);
  const TY* Y = static_cast<const TY*>(L.y);
  TZ* Z = static_cast<TZ*>(L.z);
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  bool colok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colok[q] = C + q >= 1 && C + q <= nc;
  const bool act_y = C < py, act_z = C < pz;
  const bool live = b0 < b1 && (ND == 2 || yc3 <= nc);
  // a fine "line" is one fine row (2D) or the three fine rows 2 yc3 - 1 ..
  // 2 yc3 + 1 of one fine plane (3D); share(T-index oz/oy, line, g)
  constexpr int NR = ND == 3 ? 3 : 1;
  int32_t Wm[NR][9], Wb[NR][9], Wmn[NR][9], Wbn[NR][9];
  int32_t yv[4], yn[4];
  auto load_line = [&](int64_t f, int32_t (&W)[NR][9]) {   // fine line index f
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t row = ND == 3 ? f * sf + 2 * yc3 - 1 + r : f;
      res_load(X, row * px, C, px, live && f <= nf + 1, lane, W[r]);
    }
  };
  // the share of one fine line in a coarse output with line offset o
  auto share = [&](int o, const int32_t (&W)[NR][9], int64_t (&g)[4]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int32_t* T = ND == 3 ? &t[((o + 1) * 3 + r) * 3] : &t[(o + 1) * 3];
      res_line(T, W[r], g);
    }
  };
  auto load_yv = [&](int64_t b, int32_t (&V)[4]) {
    if (HASY) ld4(Y, ((ND == 3 ? b * sc + yc3 : b)) * py + C, V, live && act_y && b <= nc);
    else V[0] = V[1] = V[2] = V[3] = 0;
  };
  // the first lines are loaded before the epilogue reads the operands'
  // metadata (they do not depend on it), so the two round trips overlap
  int32_t Wt[NR][9];
  load_line(2 * b0 - 1, Wt);                  // fine line 2 b0 - 1 (offset -1 of b0)
  load_line(2 * b0, Wm);
  load_line(2 * b0 + 1, Wb);
  load_yv(b0, yv);
  Epi<PASS, HASY> E;
  E.init(L.op);
  if (live) with_fast(E, [&](auto fast_tag) {
    constexpr int VAR = decltype(fast_tag)::value;
    int64_t carry[4] = {0, 0, 0, 0};
    share(-1, Wt, carry);
    for (int64_t I = b0; I < b1; ++I) {
      load_line(2 * I + 2, Wmn);
      load_line(2 * I + 3, Wbn);
      if (HASY) load_yv(I + 1, yn);
      int64_t g[4] = {carry[0], carry[1], carry[2], carry[3]};
      share(0, Wm, g);
      share(1, Wb, g);
      carry[0] = carry[1] = carry[2] = carry[3] = 0;
      share(-1, Wb, carry);                   // fine line 2I + 1 in coarse line I + 1
      const bool line_ok = I <= nc;
      int64_t out[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = E.template put<VAR>(g[q], yv[q], line_ok && colok[q]);
      if (PASS != kQ1 && act_z && line_ok)
        st4(Z, (ND == 3 ? I * sc + yc3 : I) * pz + C, out);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          Wm[r][k] = Wmn[r][k];
          Wb[r][k] = Wbn[r][k];
        }
      if (HASY) {
#pragma unroll
        for (int q = 0; q < 4; ++q) yv[q] = yn[q];
      }
    }
  });
  E.finish();
}

// ----------------------------------------------------------- launches ---

template <int ND, typename TX, typename TY, typename TZ, int PASS, bool HASY>
static hipError_t transfer_go(const TransferLaunch& L0, hipStream_t s) {
  TransferLaunch L = L0;
  const int rows = L.rows > 0 ? L.rows : 1;
  if (L.kind == 1) {
    const int64_t nc = L.n_out;
    const int64_t segs = (nc + 2 + 255) / 256;
    const int64_t bands = ND == 3 ? nc * ((nc + rows - 1) / rows) : (nc + rows - 1) / rows;
    if (segs * ((bands + 3) / 4) > kMaxSlotBlocks) L.op.slots = nullptr;
    hipLaunchKernelGGL((k_restrict<ND, TX, TY, TZ, PASS, HASY>),
                       dim3((unsigned)segs, (unsigned)((bands + 3) / 4)), dim3(kBlock), 0, s, L);
  } else {
    const int64_t nc = L.n_in, nf = L.n_out;
    const int64_t segs = (nf + 2 + 255) / 256;
    const int64_t nb = (nc + 1 + rows - 1) / rows;
    const int64_t bands = ND == 3 ? (nc + 1) * nb : nb;
    if (segs * ((bands + 3) / 4) > kMaxSlotBlocks) L.op.slots = nullptr;
    hipLaunchKernelGGL((k_prolong<ND, TX, TY, TZ, PASS, HASY>),
                       dim3((unsigned)segs, (unsigned)((bands + 3) / 4)), dim3(kBlock), 0, s, L);
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
