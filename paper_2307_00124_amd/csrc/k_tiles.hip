// Sub-maximal block sizes (Section 2, Remark on block size): grid vectors
// whose interior rows are split into tiles of T consecutive points along the
// fastest axis, every tile a BFP block of its own (exponent + w-bit
// mantissas). An operation forms each point's exact value and quantizes
// every output tile with the normalized floor quantization of Section 2
// (Algorithm 1's result, tile by tile).
//
// On the GPU a tile never leaves one wave: T <= 64 tiles are aligned groups
// of T lanes, larger tiles are the whole wave with T / 64 points per lane.
// The tile's largest nu is a shuffle reduction inside the wave, so an op is
// a single pass with no grid-wide reduction and no second pass — the cost
// the paper attributes to the maximal block's shared exponent.
//
// Exact range: a point's terms (alpha tap x_q at exponent alpha.e + A.exp +
// e(tile of q), beta y_p at beta.e + e(tile of p)) are summed exactly in 128
// bits after alignment to the smallest term exponent; with |alpha.m|,
// |beta.m| < 2^16, |tap| < 2^15 and |mantissa| <= 2^31 every product is
// below 2^62, and eight of them shifted by at most 60 stay below 2^126.
// A point whose term exponents spread further is counted and set to zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"
#include "device.hpp"

namespace bfpk {
namespace {

constexpr int kSpread = 60;
constexpr int kMarch = 8;   // rows (2D) or planes (3D) one wave takes in turn

struct TOp {
  const void* mant;
  const int32_t* exps;
  int64_t pitch;
  int bits;
};

struct TilesLaunch {
  int nd;
  int64_t n, ntile;      // interior points per dimension, tiles per row
  int T, K;              // tile size; points per lane (T / 64 for T > 64)
  int tsh;               // log2 T
  int64_t strips, bands, waves;
  TOp x, y;              // y: the optional second operand (mant null: none)
  void* z;
  int32_t* ze;
  int64_t pz;
  int zbits, w_out;
  int64_t am, ae;        // alpha mantissa; alpha exponent (+ stencil exponent)
  int64_t bm, be;        // beta mantissa and exponent
  // star taps: centre, x-1, x+1, slow-1, slow+1, mid-1, mid+1 (the slow
  // axis is y in 2D and z in 3D; the mid axis is y in 3D)
  int64_t taps[7];
  int32_t ct[5];         // 2D: alpha.m times the taps (centre, x-1, x+1, y-1, y+1)
  int32_t csh[6], cneg[6];  // when every |ct| and |beta.m| is a power of two:
                            // log2 and sign of ct[0..4] and beta.m
  int march;             // 2D stencil: rows one wave takes in turn
  int fast_span;         // largest exponent spread whose aligned sum fits 63 bits
  const double* f64_in;
  double* f64_out;
  int32_t* status;       // counts points beyond the exact range (or null)
};

__device__ __forceinline__ int32_t ldm(const void* p, int bits, int64_t i) {
  if (bits == 32) return static_cast<const int32_t*>(p)[i];
  if (bits == 16) return static_cast<const int16_t*>(p)[i];
  return static_cast<const int8_t*>(p)[i];
}

__device__ __forceinline__ void stm(void* p, int bits, int64_t i, int64_t v) {
  if (bits == 32) static_cast<int32_t*>(p)[i] = (int32_t)v;
  else if (bits == 16) static_cast<int16_t*>(p)[i] = (int16_t)v;
  else static_cast<int8_t*>(p)[i] = (int8_t)v;
}

// The point one lane handles for sub-step k: padded coordinates (s, m, x)
// with s the slow axis (y in 2D, z in 3D) and m the 3D middle axis y.
struct Pt {
  int64_t s, m, x;
  bool ok;
};

// The lines a wave covers: strips of 64 K columns, bands of kMarch lines
// along the slow axis (3D: one y row per wave); decomposed once per wave.
struct WaveAt {
  int64_t x0, s0, m;
};

__device__ __forceinline__ WaveAt wave_at(const TilesLaunch& L, int64_t wid) {
  const int64_t strip = wid % L.strips;
  int64_t rest = wid / L.strips;
  WaveAt w;
  w.m = 0;
  if (L.nd == 3) {
    w.m = rest % L.n + 1;
    rest /= L.n;
  }
  w.s0 = rest * kMarch + 1;
  w.x0 = strip * 64 * L.K + 1 + (threadIdx.x & 63);
  return w;
}

// band step i, lane point k
__device__ __forceinline__ Pt point_of(const TilesLaunch& L, const WaveAt& w, int i, int k) {
  Pt p;
  p.m = w.m;
  p.s = w.s0 + i;
  p.x = w.x0 + 64 * k;
  p.ok = p.x <= L.n && p.s <= L.n;
  return p;
}

__device__ __forceinline__ int64_t off(const TilesLaunch& L, int64_t pitch, int64_t s, int64_t m,
                                       int64_t x) {
  return L.nd == 3 ? (s * (L.n + 2) + m) * pitch + x : s * pitch + x;
}

// tile row of interior line (s, m)
__device__ __forceinline__ int64_t trow(const TilesLaunch& L, int64_t s, int64_t m) {
  return L.nd == 3 ? (s - 1) * L.n + (m - 1) : s - 1;
}

__device__ __forceinline__ int32_t texp(const TOp& o, const TilesLaunch& L, int64_t s, int64_t m,
                                        int64_t x) {
  return o.exps[trow(L, s, m) * L.ntile + ((x - 1) >> L.tsh)];
}

// max of nu over the lanes of a tile (T <= 64: aligned groups of T lanes;
// larger tiles: the whole wave, each lane having folded its K points)
__device__ __forceinline__ int64_t tile_max(int64_t v, int T) {
  const int span = T < 64 ? T : 64;
  for (int o = 1; o < span; o <<= 1) {
    const int64_t t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}

__device__ __forceinline__ int32_t tile_max32(int32_t v, int T) {
  const int span = T < 64 ? T : 64;
  for (int o = 1; o < span; o <<= 1) {
    const int32_t t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}

// quantize one point of a tile whose largest nu is numax: floor(v / 2^e_out)
// for v = sum 2^e0
__device__ __forceinline__ int64_t quant(__int128 sum, int64_t e0, int64_t e_out) {
  if (sum == 0) return 0;
  const int64_t sh = e_out - e0;
  if (sh >= 0) return (int64_t)(sum >> (sh > 127 ? 127 : (int)sh));
  return (int64_t)(__int128)((unsigned __int128)sum << (int)(-sh));   // fits w_out bits
}

// Count this wave's points beyond the exact range (nbad: this lane's).
__device__ __forceinline__ void count_bad(const TilesLaunch& L, int nbad) {
  if (!__ballot(nbad != 0)) return;
  const int32_t total = wave_sum32(nbad);
  if ((threadIdx.x & 63) == 0 && L.status) atomicAdd(L.status, total);
}

// Publish the output tile exponents of one line and store its points.
template <int KMAX>
__device__ __forceinline__ void finish_line(const TilesLaunch& L, const Pt (&p)[KMAX],
                                            const __int128 (&sum)[KMAX],
                                            const int64_t (&e0)[KMAX]) {
  int64_t nu = INT64_MIN;
  int64_t numax[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    numax[k] = INT64_MIN;
    if (k < L.K && p[k].ok && sum[k] != 0) numax[k] = msb128(sum[k]) + e0[k];
    nu = numax[k] > nu ? numax[k] : nu;
  }
  if (L.K == 1) nu = tile_max(numax[0], L.T);
  else nu = tile_max(nu, 64);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= L.K || !p[k].ok) continue;
    const int64_t eo = nu == INT64_MIN ? 1 - L.w_out : nu - L.w_out;
    stm(L.z, L.zbits, off(L, L.pz, p[k].s, p[k].m, p[k].x), quant(sum[k], e0[k], eo));
    if (((p[k].x - 1) & (L.T - 1)) == 0)
      L.ze[trow(L, p[k].s, p[k].m) * L.ntile + ((p[k].x - 1) >> L.tsh)] = (int32_t)eo;
  }
}

// Exact sum of the present terms aligned at their smallest exponent.
template <int NT>
__device__ __forceinline__ bool exact_sum(const int64_t (&v)[NT], const int64_t (&e)[NT],
                                          const bool (&on)[NT], __int128& sum, int64_t& e0) {
  int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (on[t]) {
      lo = e[t] < lo ? e[t] : lo;
      hi = e[t] > hi ? e[t] : hi;
    }
  sum = 0;
  e0 = lo;
  if (lo > hi) {   // no term: the value is zero
    e0 = 0;
    return true;
  }
  if (hi - lo > kSpread) return false;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (on[t] && v[t]) sum += (__int128)((unsigned __int128)(__int128)v[t] << (int)(e[t] - lo));
  return true;
}

// z = alpha A x (+ beta y) with a star stencil
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_tiles_star(const TilesLaunch L) {
  const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (wid >= L.waves) return;
  const bool hasy = L.y.mant != nullptr;
  const WaveAt wa = wave_at(L, wid);
  for (int i = 0; i < kMarch; ++i) {
    Pt p[KMAX];
    __int128 sum[KMAX];
    int64_t e0[KMAX];
    int nbad = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      p[k] = point_of(L, wa, i, k);
      sum[k] = 0;
      e0[k] = 0;
      if (k >= L.K || !p[k].ok) continue;
      const int64_t s = p[k].s, m = p[k].m, x = p[k].x;
      // neighbours: (ds, dm, dx) for centre, x-1, x+1, s-1, s+1, m-1, m+1
      const int ds[7] = {0, 0, 0, -1, 1, 0, 0};
      const int dm[7] = {0, 0, 0, 0, 0, -1, 1};
      const int dx[7] = {0, -1, 1, 0, 0, 0, 0};
      int64_t v[8], e[8];
      bool on[8];
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int64_t qs = s + ds[t], qm = m + dm[t], qx = x + dx[t];
        on[t] = L.taps[t] != 0 && (t < 5 || L.nd == 3) && qx >= 1 && qx <= L.n && qs >= 1 &&
                qs <= L.n && (L.nd == 2 || (qm >= 1 && qm <= L.n));
        v[t] = 0;
        e[t] = 0;
        if (on[t]) {
          v[t] = L.am * L.taps[t] * (int64_t)ldm(L.x.mant, L.x.bits, off(L, L.x.pitch, qs, qm, qx));
          e[t] = L.ae + texp(L.x, L, qs, qm, qx);
        }
      }
      on[7] = hasy;
      v[7] = 0;
      e[7] = 0;
      if (hasy) {
        v[7] = L.bm * (int64_t)ldm(L.y.mant, L.y.bits, off(L, L.y.pitch, s, m, x));
        e[7] = L.be + texp(L.y, L, s, m, x);
      }
      nbad += !exact_sum(v, e, on, sum[k], e0[k]);
    }
    count_bad(L, nbad);
    finish_line<KMAX>(L, p, sum, e0);
  }
}

// 2D star stencil: a wave owns a strip of 64 K columns and marches down
// L.march rows, U rows per step: the loads of a step (the next U rows of x
// with their tile exponents, the y entries and the strip's two edge columns
// of the U rows) are issued together, the rows above and below stay in
// registers, and x-neighbours come from the neighbouring lanes. When every
// lane's terms align within L.fast_span bits the exact sums are 64-bit;
// otherwise the wave takes the 128-bit form for that row.
template <int KMAX>
struct Row2 {
  int32_t m[KMAX], e[KMAX];
};

template <int KMAX, int U>
__global__ __launch_bounds__(kBlock) void k_tiles_star2d(const TilesLaunch L) {
  // wave-uniform (scalar) row and column bookkeeping
  const int64_t wid =
      (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (wid >= L.waves) return;
  const int lane = threadIdx.x & 63;
  const int64_t n = L.n, nt = L.ntile;
  const int64_t strip = wid % L.strips, band = wid / L.strips;
  const int64_t y0 = band * L.march + 1;
  const int64_t y1 = y0 + L.march - 1 < n ? y0 + L.march - 1 : n;
  const int64_t c0 = strip * 64 * L.K;   // the column left of the strip
  const int64_t cr = c0 + 64 * L.K + 1;   // the column right of it
  const bool hasy = L.y.mant != nullptr;
  const int32_t ae = (int32_t)L.ae, be = (int32_t)L.be;
  int64_t xk[KMAX], tk[KMAX];
  bool okx[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    xk[k] = c0 + 64 * k + lane + 1;
    okx[k] = xk[k] <= n;
    tk[k] = okx[k] ? (xk[k] - 1) >> L.tsh : 0;   // the lane's tile (0 off the grid)
  }
  // Branch-free row loads: a lane off the grid reads the row's first
  // element and keeps zero; rows outside the grid are zero (exponents
  // there are never used).
  auto load_row = [&](int64_t y, Row2<KMAX>& r) {
    const bool in = y >= 1 && y <= n;   // uniform
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      r.m[k] = 0;
      r.e[k] = 0;
      if (in) {
        const int32_t mv = ldm(L.x.mant, L.x.bits, y * L.x.pitch + (okx[k] ? xk[k] : 0));
        r.m[k] = okx[k] ? mv : 0;
        r.e[k] = L.x.exps[(y - 1) * nt + tk[k]];
      }
    }
  };
  Row2<KMAX> w[U + 2];   // rows y - 1 .. y + U
  load_row(y0 - 1, w[0]);
  load_row(y0, w[1]);
  for (int64_t y = y0; y <= y1; y += U) {
    int32_t ym[U][KMAX], ye[U][KMAX], eml[U], eel[U], emr[U], eer[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      load_row(y + 1 + u, w[u + 2]);
      const int64_t yy = y + u;
      const bool live = yy <= y1;   // uniform
      eml[u] = eel[u] = emr[u] = eer[u] = 0;
      if (live && c0 >= 1) {
        eml[u] = ldm(L.x.mant, L.x.bits, yy * L.x.pitch + c0);
        eel[u] = L.x.exps[(yy - 1) * nt + ((c0 - 1) >> L.tsh)];
      }
      if (live && cr <= n) {
        emr[u] = ldm(L.x.mant, L.x.bits, yy * L.x.pitch + cr);
        eer[u] = L.x.exps[(yy - 1) * nt + ((cr - 1) >> L.tsh)];
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        ym[u][k] = 0;
        ye[u][k] = 0;
        if (hasy && live) {
          const int32_t mv = ldm(L.y.mant, L.y.bits, yy * L.y.pitch + (okx[k] ? xk[k] : 0));
          ym[u][k] = okx[k] ? mv : 0;
          ye[u][k] = L.y.exps[(yy - 1) * nt + tk[k]];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t yy = y + u;
      if (yy > y1) break;   // uniform
      const Row2<KMAX>&rp = w[u], &rc = w[u + 1], &rn = w[u + 2];
      // the six terms of each point: centre, x-1, x+1, y-1, y+1, beta y. A
      // term that is absent (a ring neighbour, a zero tap, no y) has value
      // zero and takes the centre's exponent, which leaves the spread of the
      // present terms unchanged (the centre tap is nonzero on this path).
      int64_t v[KMAX][6];
      int32_t e[KMAX][6];
      bool fast_all = true;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        int32_t ml = __shfl(rc.m[k], (lane + 63) & 63), el = __shfl(rc.e[k], (lane + 63) & 63);
        int32_t mr = __shfl(rc.m[k], (lane + 1) & 63), er = __shfl(rc.e[k], (lane + 1) & 63);
        const int32_t lm = k > 0 ? __builtin_amdgcn_readlane(rc.m[k > 0 ? k - 1 : 0], 63) : eml[u];
        const int32_t le = k > 0 ? __builtin_amdgcn_readlane(rc.e[k > 0 ? k - 1 : 0], 63) : eel[u];
        const int32_t rm = k + 1 < KMAX ? __builtin_amdgcn_readlane(rc.m[k + 1 < KMAX ? k + 1 : k], 0)
                                        : emr[u];
        const int32_t re = k + 1 < KMAX ? __builtin_amdgcn_readlane(rc.e[k + 1 < KMAX ? k + 1 : k], 0)
                                        : eer[u];
        ml = lane == 0 ? lm : ml;
        el = lane == 0 ? le : el;
        mr = lane == 63 ? rm : mr;
        er = lane == 63 ? re : er;
        const int32_t ec = ae + rc.e[k];
        v[k][0] = (int64_t)L.ct[0] * rc.m[k];
        e[k][0] = ec;
        v[k][1] = (int64_t)L.ct[1] * ml;
        e[k][1] = (xk[k] > 1 && L.ct[1]) ? ae + el : ec;
        v[k][2] = (int64_t)L.ct[2] * mr;
        e[k][2] = (xk[k] < n && L.ct[2]) ? ae + er : ec;
        v[k][3] = (int64_t)L.ct[3] * rp.m[k];
        e[k][3] = (yy > 1 && L.ct[3]) ? ae + rp.e[k] : ec;
        v[k][4] = (int64_t)L.ct[4] * rn.m[k];
        e[k][4] = (yy < n && L.ct[4]) ? ae + rn.e[k] : ec;
        v[k][5] = (int64_t)L.bm * ym[u][k];
        e[k][5] = hasy ? be + ye[u][k] : ec;
        int32_t lo = e[k][0], hi = e[k][0];
#pragma unroll
        for (int t = 1; t < 6; ++t) {
          lo = e[k][t] < lo ? e[k][t] : lo;
          hi = e[k][t] > hi ? e[k][t] : hi;
        }
        fast_all &= !okx[k] || hi - lo <= L.fast_span;
      }
      if (__all(fast_all)) {
        int64_t s64[KMAX];
        int32_t e0[KMAX], nu = INT32_MIN, numax[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          int32_t lo = e[k][0];
#pragma unroll
          for (int t = 1; t < 6; ++t) lo = e[k][t] < lo ? e[k][t] : lo;
          int64_t acc = 0;
#pragma unroll
          for (int t = 0; t < 6; ++t) acc += (int64_t)((uint64_t)v[k][t] << (e[k][t] - lo));
          s64[k] = acc;
          e0[k] = lo;
          numax[k] = (okx[k] && acc != 0) ? msb64(acc) + lo : INT32_MIN;
          nu = numax[k] > nu ? numax[k] : nu;
        }
        nu = KMAX == 1 ? tile_max32(numax[0], L.T) : tile_max32(nu, 64);
        const int32_t eo = nu == INT32_MIN ? 1 - L.w_out : nu - L.w_out;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          const int32_t sh = eo - e0[k];
          const int64_t q = s64[k] == 0 ? 0
                            : sh >= 0 ? (s64[k] >> (sh > 63 ? 63 : sh))
                                      : (int64_t)((uint64_t)s64[k] << (-sh));
          if (okx[k]) {
            stm(L.z, L.zbits, yy * L.pz + xk[k], q);
            if (((xk[k] - 1) & (L.T - 1)) == 0) L.ze[(yy - 1) * nt + tk[k]] = eo;
          }
        }
      } else {
        // some point's terms spread beyond 64-bit alignment: exact 128-bit
        // sums, the absent terms excluded as such
        Pt p[KMAX];
        __int128 sum[KMAX];
        int64_t e0[KMAX];
        int nbad = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          p[k] = Pt{yy, 0, xk[k], okx[k]};
          sum[k] = 0;
          e0[k] = 0;
          const bool on[6] = {true, xk[k] > 1 && L.ct[1] != 0, xk[k] < n && L.ct[2] != 0,
                              yy > 1 && L.ct[3] != 0, yy < n && L.ct[4] != 0, hasy};
          int64_t e64[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) e64[t] = e[k][t];
          if (okx[k]) nbad += !exact_sum(v[k], e64, on, sum[k], e0[k]);
        }
        count_bad(L, nbad);
        finish_line<KMAX>(L, p, sum, e0);
      }
    }
    w[0] = w[U];
    w[1] = w[U + 1];
  }
}

// 2D star stencil for tiles of at least 4 points: a lane owns 4 consecutive
// columns (one tile holds them all), a wave a strip of 256, marching down
// L.march rows two at a time with the rows above and below in registers.
// Exponent bookkeeping (the alignment of the centre, vertical, y and the two
// edge terms) is done once per lane for its 4 points. POW2: every
// coefficient is +-2^k, so each term is a shift (no multiply).
struct Quad {
  int32_t m[4];
  int32_t e;
};

// four consecutive int32 at a 4-byte aligned address: one 16-byte access
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef i32x4 i32x4_a4 __attribute__((aligned(4)));

template <bool POW2>
__device__ __forceinline__ int64_t term(int32_t m, int32_t c, int32_t csh, int32_t cneg, int sh) {
  if (POW2) {
    const int64_t a = (int64_t)((uint64_t)(int64_t)m << (csh + sh));
    return cneg ? -a : a;
  }
  return (int64_t)((uint64_t)((int64_t)c * m) << sh);
}

template <int U, bool POW2>
__global__ __launch_bounds__(kBlock) void k_tiles_star2d4(const TilesLaunch L) {
  const int64_t wid =
      (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (wid >= L.waves) return;
  const int lane = threadIdx.x & 63;
  const int64_t n = L.n, nt = L.ntile;
  const int64_t strip = wid % L.strips, band = wid / L.strips;
  const int64_t y0 = band * L.march + 1;
  const int64_t y1 = y0 + L.march - 1 < n ? y0 + L.march - 1 : n;
  const int64_t c0 = strip * 256;          // the column left of the strip
  const int64_t x0 = c0 + 4 * lane + 1;    // the lane's first column
  const bool hasy = L.y.mant != nullptr;
  const int32_t ae = (int32_t)L.ae, be = (int32_t)L.be;
  const bool okl = x0 <= n;                // the lane holds a grid point
  const int64_t tl = okl ? (x0 - 1) >> L.tsh : 0;
  // Columns past n + 1 are read as element 0 of the row (in bounds) and
  // count as zero; n + 1 itself is the zero ring.
  auto load_quad = [&](const TOp& o, int64_t y, Quad& q) {
    const bool in = y >= 1 && y <= n;   // uniform
    q.e = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) q.m[j] = 0;
    if (!in) return;
    if (o.bits == 32) {   // uniform
      // a lane past the grid reads its row's first four elements (in
      // bounds); a quad reaching past n + 1 reads into the next row, which
      // rows 1..n always have
      const i32x4 v = *reinterpret_cast<const i32x4_a4*>(static_cast<const int32_t*>(o.mant) +
                                                         y * o.pitch + (okl ? x0 : 0));
      q.m[0] = okl ? v.x : 0;
      q.m[1] = okl && x0 + 1 <= n ? v.y : 0;
      q.m[2] = okl && x0 + 2 <= n ? v.z : 0;
      q.m[3] = okl && x0 + 3 <= n ? v.w : 0;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = x0 + j <= n;
        const int32_t v = ldm(o.mant, o.bits, y * o.pitch + (ok ? x0 + j : 0));
        q.m[j] = ok ? v : 0;
      }
    }
    q.e = o.exps[(y - 1) * nt + tl];
  };
  Quad w[U + 2];   // x rows y - 1 .. y + U
  load_quad(L.x, y0 - 1, w[0]);
  load_quad(L.x, y0, w[1]);
  for (int64_t y = y0; y <= y1; y += U) {
    Quad yq[U];
    int32_t eml[U], eel[U], emr[U], eer[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t yy = y + u;
      const bool live = yy <= y1;   // uniform
      load_quad(L.x, yy + 1, w[u + 2]);
      if (hasy && live) load_quad(L.y, yy, yq[u]);
      else {
        yq[u].e = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) yq[u].m[j] = 0;
      }
      eml[u] = eel[u] = emr[u] = eer[u] = 0;
      if (live && c0 >= 1) {
        eml[u] = ldm(L.x.mant, L.x.bits, yy * L.x.pitch + c0);
        eel[u] = L.x.exps[(yy - 1) * nt + ((c0 - 1) >> L.tsh)];
      }
      if (live && c0 + 257 <= n) {
        emr[u] = ldm(L.x.mant, L.x.bits, yy * L.x.pitch + c0 + 257);
        eer[u] = L.x.exps[(yy - 1) * nt + ((c0 + 256) >> L.tsh)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t yy = y + u;
      if (yy > y1) break;   // uniform
      const Quad &qp = w[u], &qc = w[u + 1], &qn = w[u + 2];
      // edge neighbours: the adjacent lanes' outer columns, or the strip edges
      int32_t ml = __shfl(qc.m[3], (lane + 63) & 63), el = __shfl(qc.e, (lane + 63) & 63);
      int32_t mr = __shfl(qc.m[0], (lane + 1) & 63), er = __shfl(qc.e, (lane + 1) & 63);
      ml = lane == 0 ? eml[u] : ml;
      el = lane == 0 ? eel[u] : el;
      mr = lane == 63 ? emr[u] : mr;
      er = lane == 63 ? eer[u] : er;
      // absent terms (ring neighbours, zero taps, no y) take the centre's
      // exponent; their values are zero
      const int32_t ec = ae + qc.e;
      const int32_t eL = (x0 > 1 && L.ct[1]) ? ae + el : ec;
      const int32_t eR = (x0 + 3 < n && L.ct[2]) ? ae + er : ec;
      const int32_t eU = (yy > 1 && L.ct[3]) ? ae + qp.e : ec;
      const int32_t eD = (yy < n && L.ct[4]) ? ae + qn.e : ec;
      const int32_t eY = hasy ? be + yq[u].e : ec;
      int32_t lo = ec, hi = ec;
      lo = eL < lo ? eL : lo; hi = eL > hi ? eL : hi;
      lo = eR < lo ? eR : lo; hi = eR > hi ? eR : hi;
      lo = eU < lo ? eU : lo; hi = eU > hi ? eU : hi;
      lo = eD < lo ? eD : lo; hi = eD > hi ? eD : hi;
      lo = eY < lo ? eY : lo; hi = eY > hi ? eY : hi;
      if (__all(!okl || hi - lo <= L.fast_span)) {
        const int sC = ec - lo, sL = eL - lo, sR = eR - lo, sU = eU - lo, sD = eD - lo,
                  sY = eY - lo;
        int64_t acc[4];
        int32_t nu = INT32_MIN;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int32_t lm = j > 0 ? qc.m[j > 0 ? j - 1 : 0] : ml;
          const int32_t rm = j < 3 ? qc.m[j < 3 ? j + 1 : 3] : mr;
          int64_t a = term<POW2>(qc.m[j], L.ct[0], L.csh[0], L.cneg[0], sC);
          a += term<POW2>(lm, L.ct[1], L.csh[1], L.cneg[1], j > 0 ? sC : sL);
          a += term<POW2>(rm, L.ct[2], L.csh[2], L.cneg[2], j < 3 ? sC : sR);
          a += term<POW2>(qp.m[j], L.ct[3], L.csh[3], L.cneg[3], sU);
          a += term<POW2>(qn.m[j], L.ct[4], L.csh[4], L.cneg[4], sD);
          a += term<POW2>(yq[u].m[j], (int32_t)L.bm, L.csh[5], L.cneg[5], sY);
          acc[j] = a;
          const int32_t v = (okl && x0 + j <= n && a != 0) ? msb64(a) + lo : INT32_MIN;
          nu = v > nu ? v : nu;
        }
        nu = tile_max32(nu, L.T >> 2);
        const int32_t eo = nu == INT32_MIN ? 1 - L.w_out : nu - L.w_out;
        const int32_t sh = eo - lo;
        int64_t q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          q[j] = acc[j] == 0 ? 0
                 : sh >= 0 ? (acc[j] >> (sh > 63 ? 63 : sh))
                           : (int64_t)((uint64_t)acc[j] << (-sh));
        if (L.zbits == 32 && x0 + 3 <= n) {   // a whole quad: one 16-byte store
          const i32x4 v = {(int32_t)q[0], (int32_t)q[1], (int32_t)q[2], (int32_t)q[3]};
          *reinterpret_cast<i32x4_a4*>(static_cast<int32_t*>(L.z) + yy * L.pz + x0) = v;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (x0 + j <= n) stm(L.z, L.zbits, yy * L.pz + x0 + j, q[j]);
        }
        if (okl && ((x0 - 1) & (L.T - 1)) == 0) L.ze[(yy - 1) * nt + tl] = eo;
      } else {
        // exact 128-bit sums, the absent terms excluded as such
        int32_t nu = INT32_MIN;
        __int128 sum[4];
        int64_t e0[4];
        int nbad = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t x = x0 + j;
          const int32_t lm = j > 0 ? qc.m[j > 0 ? j - 1 : 0] : ml;
          const int32_t rm = j < 3 ? qc.m[j < 3 ? j + 1 : 3] : mr;
          const int64_t v[6] = {(int64_t)L.ct[0] * qc.m[j], (int64_t)L.ct[1] * lm,
                                (int64_t)L.ct[2] * rm, (int64_t)L.ct[3] * qp.m[j],
                                (int64_t)L.ct[4] * qn.m[j], (int64_t)L.bm * yq[u].m[j]};
          const int64_t e[6] = {ec, j > 0 ? ec : ae + el, j < 3 ? ec : ae + er, ae + qp.e,
                                ae + qn.e, be + yq[u].e};
          const bool on[6] = {true, x > 1 && L.ct[1] != 0, x < n && L.ct[2] != 0,
                              yy > 1 && L.ct[3] != 0, yy < n && L.ct[4] != 0, hasy};
          sum[j] = 0;
          e0[j] = 0;
          if (x <= n) {
            nbad += !exact_sum(v, e, on, sum[j], e0[j]);
            if (sum[j] != 0) {
              const int32_t vv = (int32_t)(msb128(sum[j]) + e0[j]);
              nu = vv > nu ? vv : nu;
            }
          }
        }
        count_bad(L, nbad);
        nu = tile_max32(nu, L.T >> 2);
        const int64_t eo = nu == INT32_MIN ? 1 - L.w_out : (int64_t)nu - L.w_out;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (x0 + j <= n) stm(L.z, L.zbits, yy * L.pz + x0 + j, quant(sum[j], e0[j], eo));
        if (okl && ((x0 - 1) & (L.T - 1)) == 0) L.ze[(yy - 1) * nt + tl] = (int32_t)eo;
      }
    }
    w[0] = w[U];
    w[1] = w[U + 1];
  }
}

// z = alpha x + beta y point by point
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_tiles_axpby(const TilesLaunch L) {
  const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (wid >= L.waves) return;
  const WaveAt wa = wave_at(L, wid);
  for (int i = 0; i < kMarch; ++i) {
    Pt p[KMAX];
    __int128 sum[KMAX];
    int64_t e0[KMAX];
    int nbad = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      p[k] = point_of(L, wa, i, k);
      sum[k] = 0;
      e0[k] = 0;
      if (k >= L.K || !p[k].ok) continue;
      const int64_t s = p[k].s, m = p[k].m, x = p[k].x;
      int64_t v[2], e[2];
      bool on[2] = {true, true};
      v[0] = L.am * (int64_t)ldm(L.x.mant, L.x.bits, off(L, L.x.pitch, s, m, x));
      e[0] = L.ae + texp(L.x, L, s, m, x);
      v[1] = L.bm * (int64_t)ldm(L.y.mant, L.y.bits, off(L, L.y.pitch, s, m, x));
      e[1] = L.be + texp(L.y, L, s, m, x);
      nbad += !exact_sum(v, e, on, sum[k], e0[k]);
    }
    count_bad(L, nbad);
    finish_line<KMAX>(L, p, sum, e0);
  }
}

// Decompose a finite double as z 2^e (|z| < 2^53); false for zero and
// non-finite values (the latter also clear `finite`).
__device__ __forceinline__ bool dparts(double v, int64_t& z, int64_t& e, bool& finite) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int64_t E = (int64_t)((b >> 52) & 0x7FF);
  const int64_t F = (int64_t)(b & ((1ull << 52) - 1));
  finite = E != 0x7FF;
  if (!finite || (E == 0 && F == 0)) return false;
  const int64_t M = E ? (F | (1ll << 52)) : F;
  e = E ? E - 1075 : -1074;
  z = (b >> 63) ? -M : M;
  return true;
}

// FP64 (padded (n+2)^d array) -> tiles; non-finite inputs count as beyond
// range and become zero
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_tiles_from_f64(const TilesLaunch L) {
  const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (wid >= L.waves) return;
  const WaveAt wa = wave_at(L, wid);
  const int64_t side = L.n + 2;
  for (int i = 0; i < kMarch; ++i) {
    Pt p[KMAX];
    __int128 sum[KMAX];
    int64_t e0[KMAX];
    int nbad = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      p[k] = point_of(L, wa, i, k);
      sum[k] = 0;
      e0[k] = 0;
      if (k >= L.K || !p[k].ok) continue;
      int64_t zz, ee;
      bool fin;
      if (dparts(L.f64_in[off(L, side, p[k].s, p[k].m, p[k].x)], zz, ee, fin)) {
        sum[k] = zz;
        e0[k] = ee;
      }
      nbad += !fin;
    }
    count_bad(L, nbad);
    finish_line<KMAX>(L, p, sum, e0);
  }
}

// tiles -> FP64 (interior points of a padded (n+2)^d array): m 2^e
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_tiles_to_f64(const TilesLaunch L) {
  const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (wid >= L.waves) return;
  const WaveAt wa = wave_at(L, wid);
  const int64_t side = L.n + 2;
  for (int i = 0; i < kMarch; ++i) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const Pt p = point_of(L, wa, i, k);
      if (k >= L.K || !p.ok) continue;
      const int32_t m = ldm(L.x.mant, L.x.bits, off(L, L.x.pitch, p.s, p.m, p.x));
      const int32_t e = texp(L.x, L, p.s, p.m, p.x);
      L.f64_out[off(L, side, p.s, p.m, p.x)] = ldexp((double)m, e);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_tiles_fill(uint32_t* mant, int64_t words, int32_t* exps,
                                                       int64_t ntiles, int32_t e) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < words + ntiles;
       i += (int64_t)gridDim.x * kBlock) {
    if (i < words) mant[i] = 0;
    else exps[i - words] = e;
  }
}

// launch kernel family F with the points-per-lane instantiation T / 64
template <typename F>
hipError_t launch_k(const TilesLaunch& L, F&& pick) {
  const unsigned blocks = (unsigned)((L.waves + kBlock / 64 - 1) / (kBlock / 64));
  if (L.K == 1) pick(std::integral_constant<int, 1>(), blocks);
  else if (L.K == 2) pick(std::integral_constant<int, 2>(), blocks);
  else pick(std::integral_constant<int, 4>(), blocks);
  return hipGetLastError();
}

int bitlen_host(int64_t v) {
  uint64_t u = (uint64_t)(v < 0 ? -v : v);
  int b = 0;
  while (u) {
    ++b;
    u >>= 1;
  }
  return b;
}

int check_tiles(const bfp_tiles* t, const char* name) {
  if (!t) return fail(BFP_EINVAL, "%s is NULL", name);
  if (!t->mant || !t->exps) return fail(BFP_EINVAL, "%s: NULL device pointer", name);
  if (t->ndim != 2 && t->ndim != 3) return fail(BFP_ESHAPE, "%s: ndim must be 2 or 3", name);
  if (t->n < 1) return fail(BFP_ESHAPE, "%s: n must be >= 1", name);
  if (t->T < 1 || t->T > 256 || (t->T & (t->T - 1)))
    return fail(BFP_ESHAPE, "%s: the tile size must be a power of two in 1..256", name);
  if (t->storage_bits != 8 && t->storage_bits != 16 && t->storage_bits != 32)
    return fail(BFP_EWIDTH, "%s: storage_bits must be 8, 16 or 32", name);
  if (t->w < 1 || t->w > t->storage_bits)
    return fail(BFP_EWIDTH, "%s: width must be in 1..storage_bits", name);
  if (t->pitch < t->n + 2 || (t->pitch * (t->storage_bits / 8)) % 16)
    return fail(BFP_ESHAPE, "%s: pitch must hold n + 2 elements and be a multiple of 16 bytes", name);
  return BFP_OK;
}

int same_tiling(const bfp_tiles* a, const bfp_tiles* b) {
  if (a->ndim != b->ndim || a->n != b->n || a->T != b->T)
    return fail(BFP_ESHAPE, "operands must share ndim, n and the tile size");
  return BFP_OK;
}

TilesLaunch base_launch(const bfp_tiles* shape) {
  TilesLaunch L;
  std::memset(&L, 0, sizeof L);
  L.nd = shape->ndim;
  L.n = shape->n;
  L.T = shape->T;
  L.K = shape->T > 64 ? shape->T / 64 : 1;
  L.ntile = (L.n + L.T - 1) / L.T;
  L.tsh = 0;
  while ((1 << L.tsh) < L.T) ++L.tsh;
  L.strips = (L.n + 64 * L.K - 1) / (64 * L.K);
  L.bands = (L.n + kMarch - 1) / kMarch;
  L.waves = L.strips * L.bands * (L.nd == 3 ? L.n : 1);
  return L;
}

TOp op_of(const bfp_tiles* t) { return TOp{t->mant, t->exps, t->pitch, t->storage_bits}; }

void set_out(TilesLaunch& L, bfp_tiles* z, int32_t* status) {
  L.z = z->mant;
  L.ze = z->exps;
  L.pz = z->pitch;
  L.zbits = z->storage_bits;
  L.w_out = z->w;
  L.status = status;
}

int scalar_ok(const bfp_scalar* a, const char* name) {
  if (!a) return fail(BFP_EINVAL, "%s is NULL", name);
  if (a->m <= -(1 << 16) || a->m >= (1 << 16))
    return fail(BFP_EWIDTH, "%s: |mantissa| must be below 2^16 for tiled operands", name);
  if (a->exp < -(1ll << 28) || a->exp > (1ll << 28))
    return fail(BFP_EINVAL, "%s: exponent out of range (|exp| <= 2^28)", name);
  return BFP_OK;
}

}  // namespace
}  // namespace bfpk

using namespace bfpk;

extern "C" {

int bfp_tiles_layout(int ndim, int n, int T, int storage_bits, int64_t* pitch, size_t* mant_bytes,
                     size_t* exp_bytes) {
  if (T < 1 || T > 256 || (T & (T - 1)))
    return fail(BFP_ESHAPE, "the tile size must be a power of two in 1..256");
  int rc = bfp_layout(ndim, n, storage_bits, pitch, mant_bytes);
  if (rc) return rc;
  const int64_t rows = ndim == 3 ? (int64_t)n * n : n;
  if (exp_bytes) *exp_bytes = (size_t)(rows * ((n + T - 1) / T)) * sizeof(int32_t);
  return BFP_OK;
}

int bfp_tiles_init(const bfp_tiles* t, void* stream) {
  int rc = check_tiles(t, "t");
  if (rc) return rc;
  const int64_t side = t->n + 2;
  const int64_t rows = t->ndim == 3 ? side * side : side;
  const int64_t words = t->pitch * rows * (t->storage_bits / 8) / 4;
  const int64_t trows = t->ndim == 3 ? (int64_t)t->n * t->n : t->n;
  const int64_t ntiles = trows * ((t->n + t->T - 1) / t->T);
  const int64_t total = words + ntiles;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_tiles_fill, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream,
                     static_cast<uint32_t*>(t->mant), words, t->exps, ntiles, 1 - t->w);
  return hip_check(hipGetLastError(), "bfp_tiles_init");
}

int bfp_tiles_from_f64(const double* x_dev, bfp_tiles* out, int32_t* status_dev, void* stream) {
  if (!x_dev) return fail(BFP_EINVAL, "x is NULL");
  int rc = check_tiles(out, "out");
  if (rc) return rc;
  TilesLaunch L = base_launch(out);
  set_out(L, out, status_dev);
  L.f64_in = x_dev;
  hipStream_t s = (hipStream_t)stream;
  return hip_check(launch_k(L, [&](auto k, unsigned blocks) {
                     hipLaunchKernelGGL((k_tiles_from_f64<decltype(k)::value>), dim3(blocks),
                                        dim3(kBlock), 0, s, L);
                   }),
                   "bfp_tiles_from_f64");
}

int bfp_tiles_to_f64(const bfp_tiles* in, double* x_dev, void* stream) {
  if (!x_dev) return fail(BFP_EINVAL, "x is NULL");
  int rc = check_tiles(in, "in");
  if (rc) return rc;
  TilesLaunch L = base_launch(in);
  L.x = op_of(in);
  L.f64_out = x_dev;
  hipStream_t s = (hipStream_t)stream;
  return hip_check(launch_k(L, [&](auto k, unsigned blocks) {
                     hipLaunchKernelGGL((k_tiles_to_f64<decltype(k)::value>), dim3(blocks),
                                        dim3(kBlock), 0, s, L);
                   }),
                   "bfp_tiles_to_f64");
}

int bfp_tiles_stencil_apply(const bfp_stencil* A, const bfp_tiles* x, const bfp_scalar* alpha,
                            const bfp_scalar* beta, const bfp_tiles* y, bfp_tiles* z,
                            int32_t* status_dev, void* stream) {
  if (!A) return fail(BFP_EINVAL, "A is NULL");
  int rc;
  if ((rc = check_tiles(x, "x")) || (rc = check_tiles(z, "z")) || (rc = same_tiling(x, z)))
    return rc;
  if (y && ((rc = check_tiles(y, "y")) || (rc = same_tiling(x, y)))) return rc;
  if ((rc = scalar_ok(alpha, "alpha"))) return rc;
  if (y && (rc = scalar_ok(beta, "beta"))) return rc;
  if (A->exp < -(1ll << 28) || A->exp > (1ll << 28)) return fail(BFP_EINVAL, "A: exponent out of range");
  if (A->kind != BFP_STENCIL_A || A->ndim != x->ndim)
    return fail(BFP_EINVAL, "tiled operands take a same-grid stencil of their dimension");
  if (z->mant == x->mant || z->exps == x->exps)
    return fail(BFP_EINVAL, "z must not alias x (neighbours are read after other tiles are written)");
  // star taps only: centre, x-1, x+1, slow-1, slow+1, mid-1, mid+1
  const int idx2[7] = {4, 3, 5, 1, 7, -1, -1};
  const int idx3[7] = {13, 12, 14, 4, 22, 10, 16};
  const int* idx = A->ndim == 2 ? idx2 : idx3;
  const int ntaps = A->ndim == 2 ? 9 : 27;
  int64_t taps[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < ntaps; ++k) {
    bool star = false;
    for (int t = 0; t < 7; ++t)
      if (idx[t] == k) {
        star = true;
        taps[t] = A->taps[k];
      }
    if (!star && A->taps[k] != 0) return fail(BFP_EINVAL, "tiled operands take star stencils only");
  }
  for (int t = 0; t < 7; ++t)
    if (taps[t] <= -(1 << 15) || taps[t] >= (1 << 15))
      return fail(BFP_EWIDTH, "stencil taps must be below 2^15 in magnitude");
  TilesLaunch L = base_launch(x);
  L.x = op_of(x);
  if (y) {
    L.y = op_of(y);
    L.bm = beta->m;
    L.be = beta->exp;
  }
  set_out(L, z, status_dev);
  L.am = alpha->m;
  L.ae = alpha->exp + A->exp;
  for (int t = 0; t < 7; ++t) L.taps[t] = taps[t];
  hipStream_t s = (hipStream_t)stream;
  if (x->ndim == 3 || taps[0] == 0)   // 3D, or a stencil without centre tap
    return hip_check(launch_k(L, [&](auto k, unsigned blocks) {
                       hipLaunchKernelGGL((k_tiles_star<decltype(k)::value>), dim3(blocks),
                                          dim3(kBlock), 0, s, L);
                     }),
                     "bfp_tiles_stencil_apply");
  // 2D: coefficient products, the 64-bit span, the march length
  int vb = 0;
  for (int t = 0; t < 5; ++t) {
    L.ct[t] = (int32_t)(alpha->m * taps[t]);
    vb = std::max(vb, bitlen_host(L.ct[t]) + 31);
  }
  if (y) vb = std::max(vb, bitlen_host(beta->m) + 31);
  L.fast_span = 59 - vb;   // six terms below 2^(vb + span) sum below 2^(vb + span + 3)
  if (L.T >= 4) {
    // 4 columns per lane, strips of 256, two rows per step
    bool pow2 = true;
    for (int t = 0; t < 6; ++t) {
      const int64_t c = t < 5 ? L.ct[t] : (y ? beta->m : 0);
      const uint64_t a = (uint64_t)(c < 0 ? -c : c);
      L.cneg[t] = c < 0;
      L.csh[t] = a ? bitlen_host((int64_t)a) - 1 : 0;
      // a zero coefficient (of a term that exists) needs the multiply form
      if ((a & (a - 1)) || (!a && (t < 5 || y))) pow2 = false;
    }
    L.strips = (L.n + 255) / 256;
    L.march = 2;
    if (tiles_rows() >= 2) L.march = tiles_rows() & ~1;
    else
      while (L.march < 64 && L.strips * ((L.n + 2 * L.march - 1) / (2 * L.march)) >= 8192)
        L.march *= 2;
    L.bands = (L.n + L.march - 1) / L.march;
    L.waves = L.strips * L.bands;
    const unsigned blocks = (unsigned)((L.waves + kBlock / 64 - 1) / (kBlock / 64));
    if (pow2) hipLaunchKernelGGL((k_tiles_star2d4<2, true>), dim3(blocks), dim3(kBlock), 0, s, L);
    else hipLaunchKernelGGL((k_tiles_star2d4<2, false>), dim3(blocks), dim3(kBlock), 0, s, L);
    return hip_check(hipGetLastError(), "bfp_tiles_stencil_apply");
  }
  // rows per step: 4 / K (a step's loads in flight together), march a
  // multiple of it while the grid keeps at least 8192 waves
  const int U = 4 / L.K;
  L.march = U;
  while (L.march < 32 && L.strips * ((L.n + 2 * L.march - 1) / (2 * L.march)) >= 8192) L.march *= 2;
  L.bands = (L.n + L.march - 1) / L.march;
  L.waves = L.strips * L.bands;
  return hip_check(launch_k(L, [&](auto k, unsigned blocks) {
                     constexpr int KM = decltype(k)::value;
                     hipLaunchKernelGGL((k_tiles_star2d<KM, 4 / KM>), dim3(blocks), dim3(kBlock),
                                        0, s, L);
                   }),
                   "bfp_tiles_stencil_apply");
}

int bfp_tiles_axpby(const bfp_scalar* alpha, const bfp_tiles* x, const bfp_scalar* beta,
                    const bfp_tiles* y, bfp_tiles* z, int32_t* status_dev, void* stream) {
  int rc;
  if ((rc = check_tiles(x, "x")) || (rc = check_tiles(y, "y")) || (rc = check_tiles(z, "z")) ||
      (rc = same_tiling(x, y)) || (rc = same_tiling(x, z)))
    return rc;
  if ((rc = scalar_ok(alpha, "alpha")) || (rc = scalar_ok(beta, "beta"))) return rc;
  TilesLaunch L = base_launch(x);
  L.x = op_of(x);
  L.y = op_of(y);
  set_out(L, z, status_dev);
  L.am = alpha->m;
  L.ae = alpha->exp;
  L.bm = beta->m;
  L.be = beta->exp;
  hipStream_t s = (hipStream_t)stream;
  return hip_check(launch_k(L, [&](auto k, unsigned blocks) {
                     hipLaunchKernelGGL((k_tiles_axpby<decltype(k)::value>), dim3(blocks),
                                        dim3(kBlock), 0, s, L);
                   }),
                   "bfp_tiles_axpby");
}

}  // extern "C"
