// The V-cycle's relaxation from zero and the residual after it, fused (2D):
//   y = Q(c2 A r + c1 r)   (relaxation, nnqcomp)
//   s = Q(A y - r)         (residual, nnqcomp)
// In nnqcomp both output exponents come from the Table 1 estimates, which
// read only r's metadata, so a wave can quantize a row of y and then, from
// three rows of y it holds in registers, a row of s: r is read once, y is
// written once and never read back, and both land in one launch. Every
// value equals what the two separate star launches store (the same exact
// row sums, the same epilogue); the metadata of both outputs (exponent,
// max, min, saturations) is reduced through per-block slots and published
// by the block that finishes last.
//
// Layout: a wave owns 256 columns (4 per lane) of rows [r0, r1) of y and s.
// It marches down its rows keeping r rows k..k+2 and y rows k-1..k+1 in
// registers: at row k it quantizes y row k + 1 and then s row k. The rows
// of y just outside the band (r0 - 1 and r1) and the two columns beside the
// wave's segment are computed again from r (never stored or counted), so
// no wave waits for another.
#include "epilogue.hpp"
#include "vcycle.hpp"

namespace bfpk {

namespace {

// Metadata of the residual's operands: its x is the relaxation's output,
// whose exponent this launch fixes (known before any value is computed).
struct FusedMeta {
  PtrMeta m;
  int64_t ey;
  __device__ __forceinline__ int64_t operator()(int k, int f) const {
    return (k == kOpX && f == kMetaExp) ? ey : m(k, f);
  }
};

// One row of r: the lane's 4 columns c..c+3 and, for the wave-edge lanes,
// the two columns beyond the segment on their side (lane 0: c - 1, c - 2;
// lane 63: c + 4, c + 5). Rows outside 0..n+1 and columns outside the
// pitch read as 0.
struct RRow {
  int32_t v[4];
  int32_t e, e2;
};

__device__ __forceinline__ void rr_load(const int32_t* R, int64_t k, int64_t n, int64_t pr,
                                        int64_t c, int lane, bool live, RRow& o) {
  const bool ok = live && k >= 0 && k <= n + 1;
  ld4(R, k * pr + c, o.v, ok && c < pr);
  const bool edge = lane == 0 || lane == 63;
  const int64_t ce = lane == 0 ? c - 1 : c + 4, ce2 = lane == 0 ? c - 2 : c + 5;
  o.e = ld1(R, k * pr + ce, ok && edge && ce >= 0 && ce < pr);
  o.e2 = ld1(R, k * pr + ce2, ok && edge && ce2 >= 0 && ce2 < pr);
}

template <class E>
__device__ __forceinline__ int32_t clamped(const E& e, int64_t v) {
  return (int32_t)(v < e.lo ? e.lo : (v > e.hi ? e.hi : v));
}

// y row j from r rows j - 1 (up), j (cur), j + 1 (dn): the lane's 4 values
// and the value at its wave-edge column (lane 0: c - 1, lane 63: c + 4).
// count: the row is the wave's own (its values are counted in the
// metadata); other rows are recomputed halo rows, not counted.
template <int VAR, class E>
__device__ __forceinline__ void y_row(E& Ey, const int32_t (&t)[5], const RRow& up,
                                      const RRow& cur, const RRow& dn, int64_t j, int64_t n,
                                      int64_t c, int lane, bool count, int32_t (&y)[4],
                                      int32_t& ye) {
  const bool row_in = j >= 1 && j <= n;
  int32_t left = __shfl_up(cur.v[3], 1, 64);
  int32_t right = __shfl_down(cur.v[0], 1, 64);
  if (lane == 0) left = cur.e;
  if (lane == 63) right = cur.e;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t xl = q ? cur.v[q - 1] : left;
    const int32_t xr = q < 3 ? cur.v[q + 1] : right;
    const int64_t g = (int64_t)t[0] * cur.v[q] + (int64_t)t[1] * xl + (int64_t)t[2] * xr +
                      (int64_t)t[3] * up.v[q] + (int64_t)t[4] * dn.v[q];
    const bool in = row_in && c + q >= 1 && c + q <= n;
    if (count) y[q] = (int32_t)Ey.template put<VAR>(g, cur.v[q], in);
    else y[q] = in ? clamped(Ey, Ey.template value<VAR>(g, cur.v[q])) : 0;
  }
  // the wave-edge column ce: lane 0 reads r at c - 2, c - 1, c; lane 63 at
  // c + 3, c + 4, c + 5 (the other lanes compute a value they never use)
  const int64_t ce = lane == 0 ? c - 1 : c + 4;
  const int32_t el = lane == 0 ? cur.e2 : cur.v[3];
  const int32_t er = lane == 0 ? cur.v[0] : cur.e2;
  const int64_t ge = (int64_t)t[0] * cur.e + (int64_t)t[1] * el + (int64_t)t[2] * er +
                     (int64_t)t[3] * up.e + (int64_t)t[4] * dn.e;
  const bool ein = row_in && ce >= 1 && ce <= n;
  ye = ein ? clamped(Ey, Ey.template value<VAR>(ge, cur.e)) : 0;
}

// s row k from y rows k - 1, k, k + 1 (and y's wave-edge values of row k)
// and r row k (the y operand of the residual).
template <int VAR, class E>
__device__ __forceinline__ void s_row(E& Es, const int32_t (&t)[5], const int32_t (&yu)[4],
                                      const int32_t (&yc)[4], int32_t yce, const int32_t (&yd)[4],
                                      const RRow& r, bool row_ok, const bool (&colok)[4],
                                      int lane, int64_t (&out)[4]) {
  int32_t left = __shfl_up(yc[3], 1, 64);
  int32_t right = __shfl_down(yc[0], 1, 64);
  if (lane == 0) left = yce;
  if (lane == 63) right = yce;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t xl = q ? yc[q - 1] : left;
    const int32_t xr = q < 3 ? yc[q + 1] : right;
    const int64_t g = (int64_t)t[0] * yc[q] + (int64_t)t[1] * xl + (int64_t)t[2] * xr +
                      (int64_t)t[3] * yu[q] + (int64_t)t[4] * yd[q];
    out[q] = Es.template put<VAR>(g, r.v[q], row_ok && colok[q]);
  }
}

__device__ __forceinline__ void st4i(int32_t* base, int64_t off, const int32_t (&v)[4]) {
  const int64_t w[4] = {v[0], v[1], v[2], v[3]};
  st4(base, off, w);
}

// The two outputs' reductions: per-block partials of y (slots [0, 2 nblk))
// and s (slots [2 nblk, 4 nblk)), one ticket (on y's metadata), and the last
// block publishes both.
template <class EA, class EB>
__device__ __forceinline__ void finish_two(const EA& A, const EB& B, int64_t* slots) {
  __shared__ int32_t red[6][kBlock / 64];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int32_t v[6] = {wave_max32(A.tmax), wave_min32(A.tmin), wave_sum32(A.tsat),
                        wave_max32(B.tmax), wave_min32(B.tmin), wave_sum32(B.tsat)};
  if ((tid & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) red[i][tid >> 6] = v[i];
  }
  __syncthreads();
  const unsigned nblk = gridDim.x;
  int64_t* za = A.zm;
  int64_t* zb = B.zm;
  if (tid == 0) {
    int32_t bmax[2], bmin[2];
    int64_t bsat[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      bmax[o] = red[3 * o][0];
      bmin[o] = red[3 * o + 1][0];
      bsat[o] = red[3 * o + 2][0];
      for (int i = 1; i < kBlock / 64; ++i) {
        bmax[o] = red[3 * o][i] > bmax[o] ? red[3 * o][i] : bmax[o];
        bmin[o] = red[3 * o + 1][i] < bmin[o] ? red[3 * o + 1][i] : bmin[o];
        bsat[o] += red[3 * o + 2][i];
      }
    }
    if (nblk == 1) {
      za[kMetaMax] = bmax[0];
      za[kMetaMin] = bmin[0];
      za[kMetaSat] = bsat[0];
      za[kMetaExp] = A.R.eo;
      zb[kMetaMax] = bmax[1];
      zb[kMetaMin] = bmin[1];
      zb[kMetaSat] = bsat[1];
      zb[kMetaExp] = B.R.eo;
      s_last = 0;
    } else {
      const unsigned blk = blockIdx.x;
      int64_t r = 0;
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const uint64_t packed = ((uint64_t)(uint32_t)bmax[o] << 32) | (uint32_t)bmin[o];
        int64_t* sl = slots + 2 * (int64_t)nblk * o;
        r ^= axch(&sl[2 * blk], (int64_t)packed) ^ axch(&sl[2 * blk + 1], bsat[o]);
      }
      s_last = take_ticket(za, r);
    }
  }
  __syncthreads();
  if (!s_last || tid >= 64) return;
  int32_t mx[2] = {0, 0}, mn[2] = {0, 0};
  int64_t st[2] = {0, 0};
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    int64_t* sl = slots + 2 * (int64_t)nblk * o;
    for (unsigned k = tid; k < nblk; k += 64) {
      const uint64_t p = (uint64_t)axch(&sl[2 * k], 0);
      const int32_t hmax = (int32_t)(uint32_t)(p >> 32), hmin = (int32_t)(uint32_t)p;
      mx[o] = hmax > mx[o] ? hmax : mx[o];
      mn[o] = hmin < mn[o] ? hmin : mn[o];
      st[o] += axch(&sl[2 * k + 1], 0);
    }
    mx[o] = wave_max32(mx[o]);
    mn[o] = wave_min32(mn[o]);
    // two 32-bit DPP sums (low 24 bits and the rest; exact below 2^55)
    const int32_t slo = wave_sum32((int32_t)(st[o] & 0xFFFFFF)), shi = wave_sum32((int32_t)(st[o] >> 24));
    st[o] = ((int64_t)shi << 24) + slo;
  }
  if (tid == 0) {
    axch(&za[kMetaTicket], 0);
    za[kMetaMax] = mx[0];
    za[kMetaMin] = mn[0];
    za[kMetaSat] = st[0];
    za[kMetaExp] = A.R.eo;
    zb[kMetaMax] = mx[1];
    zb[kMetaMin] = mn[1];
    zb[kMetaSat] = st[1];
    zb[kMetaExp] = B.R.eo;
  }
}

// dispatch id -> tile: XCD k (dispatch ids congruent to k mod 8) receives a
// contiguous run of tiles, so bands that share halo rows of r mostly run
// on one XCD and read them from its L2
__device__ __forceinline__ int64_t rr_tile(int64_t id, int64_t nblk) {
  const int64_t q = nblk / 8, rem = nblk % 8;
  const int64_t k = id % 8, j = id / 8;
  return k * q + (k < rem ? k : rem) + j;
}

__global__ __launch_bounds__(kBlock) void k_relax_res2d(const RelaxResLaunch P) {
  const int lane = threadIdx.x & 63;
  const int64_t n = P.relax.n;
  const int64_t pr = P.relax.px, py = P.relax.pz, ps = P.res.pz;
  const int rows = P.rows;
  const int64_t segs = (n + 2 + 255) / 256, bands = (n + rows - 1) / rows;
  const int64_t w = rr_tile(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t seg = w % segs, band = w / segs;
  const bool live = band < bands;
  const int64_t c = seg * 256 + lane * 4;
  const int64_t r0 = 1 + band * rows;
  const int64_t r1 = r0 + rows < n + 1 ? r0 + rows : n + 1;
  const int32_t* R = static_cast<const int32_t*>(P.relax.x);
  int32_t* Yo = static_cast<int32_t*>(P.relax.z);
  int32_t* So = static_cast<int32_t*>(P.res.z);
  int32_t ta[5], tb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    ta[k] = P.relax.taps[k];
    tb[k] = P.res.taps[k];
  }
  bool colok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colok[q] = c + q >= 1 && c + q <= n;
  const bool act_y = c < py, act_s = c < ps;
  // r rows r0 - 2 .. r0 + 2, issued before the metadata is read
  RRow a, b, r0w, r1w, r2w;
  rr_load(R, r0 - 2, n, pr, c, lane, live, a);
  rr_load(R, r0 - 1, n, pr, c, lane, live, b);
  rr_load(R, r0, n, pr, c, lane, live, r0w);
  rr_load(R, r0 + 1, n, pr, c, lane, live, r1w);
  rr_load(R, r0 + 2, n, pr, c, lane, live, r2w);
  Epi<kOut, true> Ey, Es;
  Ey.init(P.relax.op);
  Es.init(P.res.op, FusedMeta{ptr_meta(P.res.op), Ey.R.eo});
  if (live) with_fast(Ey, [&](auto ytag) {
    constexpr int VY = decltype(ytag)::value;
    with_fast(Es, [&](auto stag) {
      constexpr int VS = decltype(stag)::value;
      int32_t ym[4], yc[4], yp[4], yem, yec, yep;
      y_row<VY>(Ey, ta, a, b, r0w, r0 - 1, n, c, lane, false, ym, yem);
      y_row<VY>(Ey, ta, b, r0w, r1w, r0, n, c, lane, true, yc, yec);
      if (act_y) st4i(Yo, r0 * py + c, yc);
      RRow q0 = r0w, q1 = r1w, q2 = r2w;   // r rows k, k + 1, k + 2
      for (int64_t k = r0; k < r1; ++k) {
        RRow qn;
        rr_load(R, k + 3, n, pr, c, lane, true, qn);
        const bool own = k + 1 < r1;
        y_row<VY>(Ey, ta, q0, q1, q2, k + 1, n, c, lane, own, yp, yep);
        if (own && act_y) st4i(Yo, (k + 1) * py + c, yp);
        int64_t out[4];
        s_row<VS>(Es, tb, ym, yc, yec, yp, q0, k <= n, colok, lane, out);
        if (act_s) st4(So, k * ps + c, out);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ym[q] = yc[q];
          yc[q] = yp[q];
        }
        yem = yec;
        yec = yep;
        q0 = q1;
        q1 = q2;
        q2 = qn;
      }
      (void)yem;
    });
  });
  finish_two(Ey, Es, P.slots);
}

}  // namespace

bool relax_res_fits(const StarLaunch& a, const StarLaunch& b) {
  return a.ndim == 2 && b.ndim == 2 && a.n == b.n && a.n >= 1 && a.op.mode == kModeSat &&
         b.op.mode == kModeSat && a.op.has_y && b.op.has_y && a.y_is_x && a.x == a.y &&
         b.x == a.z && b.y == a.x && a.xbits == 32 && a.zbits == 32 && b.xbits == 32 &&
         b.ybits == 32 && b.zbits == 32 && a.px % 4 == 0 && a.pz % 4 == 0 && b.pz % 4 == 0 &&
         b.px == a.pz && b.py == a.px && a.op.diag == nullptr && b.op.diag == nullptr;
}

int64_t relax_res_blocks(int64_t n, int rows) {
  const int64_t segs = (n + 2 + 255) / 256, bands = (n + rows - 1) / rows;
  return (segs * bands + kBlock / 64 - 1) / (kBlock / 64);
}

hipError_t launch_relax_res(const RelaxResLaunch& L, hipStream_t s) {
  if (!relax_res_fits(L.relax, L.res) || L.rows < 1 || !L.slots) return hipErrorInvalidValue;
  const int64_t blocks = relax_res_blocks(L.relax.n, L.rows);
  if (blocks < 1 || 2 * blocks > kMaxSlotBlocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relax_res2d, dim3((unsigned)blocks), dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

}  // namespace bfpk
