// Coarse-level executor: one workgroup of kExecThreads threads runs a
// recorded list of BFP operations (star stencils, grid transfers, pointwise
// ops, zero fills) one after the other, with a workgroup barrier between
// them. Each operation computes exactly what its stand-alone kernel computes
// — the same exact row sums and the same epilogue (the generic exact
// combine) — and publishes its metadata from a workgroup reduction, so a
// whole coarse V-cycle, or the coarse levels of FMG, cost one launch instead
// of one or two launches per operation.
//
// Storage types are read at run time: loads fetch the aligned 32-bit word
// holding an element and extract it, which keeps every load of a batch
// branch-free; stores branch (uniformly) on the type.
//
// Latency is what matters at this size, so the executor keeps the
// metadata of every block the program touches in LDS (loaded at the start,
// written back at the end) and prefetches each recorded op into an LDS
// double buffer while the previous one runs: per op, the only global
// round trips left are the data loads and the store acknowledgements.
#include "epilogue.hpp"

namespace bfpk {

namespace {

constexpr int kExWaves = kExecThreads / 64;

// Pointers read from the recorded ops are generic; the data all lives in
// global memory, and saying so keeps loads and stores off the flat path
// (whose waits would also cover the LDS traffic of the executor).
#define BFP_GLOBAL __attribute__((address_space(1)))

struct Src {
  const BFP_GLOBAL char* p;
  int sh;     // log2 of the element size in bytes
  int bits;
};

__device__ __forceinline__ Src src_of(const void* p, int bits) {
  return Src{(const BFP_GLOBAL char*)p, bits == 32 ? 2 : (bits == 16 ? 1 : 0), bits};
}

// element i, sign-extended from its storage width
__device__ __forceinline__ int32_t ldx(const Src& s, int64_t i) {
  const int64_t off = i << s.sh;
  const uint32_t word = *(const BFP_GLOBAL uint32_t*)(s.p + (off & ~(int64_t)3));
  const int at = (int)(off & 3) * 8;
  return (int32_t)(word << (32 - s.bits - at)) >> (32 - s.bits);
}

__device__ __forceinline__ void stv(void* p, int bits, int64_t i, int64_t v) {
  if (bits == 32) ((BFP_GLOBAL int32_t*)p)[i] = (int32_t)v;
  else if (bits == 16) ((BFP_GLOBAL int16_t*)p)[i] = (int16_t)v;
  else ((BFP_GLOBAL int8_t*)p)[i] = (int8_t)v;
}

typedef int64_t MetaRow[kExMetaF];

// Operand metadata read from the LDS mirror by slot.
struct LdsMeta {
  MetaRow* lm;
  int s[5];
  __device__ __forceinline__ int64_t operator()(int k, int f) const { return lm[s[k]][f]; }
};

__device__ __forceinline__ LdsMeta lds_meta(MetaRow* lm, const int16_t* slot) {
  LdsMeta m;
  m.lm = lm;
  m.s[kOpX] = slot[0];
  m.s[kOpY] = slot[1] >= 0 ? slot[1] : slot[0];
  m.s[kOpZ] = slot[2];
  m.s[kOpGa] = slot[3] >= 0 ? slot[3] : 0;
  m.s[kOpGb] = slot[4] >= 0 ? slot[4] : 0;
  return m;
}

// Workgroup reductions: per-wave partials (DPP) in LDS, then wave 0
// reduces them and lane 0 publishes the result in the output's LDS row.
template <int PASS, bool HASY>
__device__ __forceinline__ void ex_finish(const Epi<PASS, HASY>& E, MetaRow& zm) {
  __shared__ int32_t red[3][kExWaves];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (PASS == kQ1) {
    const int32_t m = wave_max32((int32_t)E.tmu);
    if (lane == 0) red[0][wave] = m;
    __syncthreads();
    if (wave == 0) {
      const int32_t b = wave_max32(lane < kExWaves ? red[0][lane] : 1);
      if (lane == 0) zm[kMetaMu] = b;
    }
  } else {
    const int32_t a = wave_max32(E.tmax), b = wave_min32(E.tmin), c = wave_sum32(E.tsat);
    if (lane == 0) {
      red[0][wave] = a;
      red[1][wave] = b;
      red[2][wave] = c;
    }
    __syncthreads();
    if (wave == 0) {
      const bool in = lane < kExWaves;
      const int32_t mx = wave_max32(in ? red[0][lane] : 0);
      const int32_t mn = wave_min32(in ? red[1][lane] : 0);
      const int32_t st = wave_sum32(in ? red[2][lane] : 0);
      if (lane == 0) {
        zm[kMetaMax] = mx;
        zm[kMetaMin] = mn;
        zm[kMetaSat] = st;
        zm[kMetaExp] = E.R.eo;
      }
    }
  }
  __syncthreads();
}

// Visit every interior point (z, y, x) of an n^ND output grid: the exact
// value g = gather(z, y, x), the optional y entry, the epilogue and the store.
// Points are enumerated on a 2^lg >= n padded index space; a padding slot
// becomes the interior point (1, 1, 1), which keeps every address in bounds,
// and is neither stored nor counted.
template <int ND, int PASS, bool HASY, int U, typename Gather>
__device__ __forceinline__ void ex_loop(const OpArgs& op, const LdsMeta& ma, int n,
                                        const void* yp, int ybits, int64_t py, void* zp,
                                        int zbits, int64_t pz, Gather&& gather) {
  Epi<PASS, HASY> E;
  E.init(op, ma);
  const Src ys = src_of(yp, ybits);
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const int M = (1 << lg) - 1;
  const int tot = ND == 3 ? 1 << (3 * lg) : 1 << (2 * lg);
  const int64_t side = n + 2;
  for (int i0 = threadIdx.x; i0 < tot; i0 += U * kExecThreads) {
    int64_t g[U], zo[U];
    int32_t yv[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kExecThreads;
      int x = (i & M) + 1, y = ((i >> lg) & M) + 1, z = ND == 3 ? (i >> (2 * lg)) + 1 : 0;
      ok[u] = i < tot && x <= n && y <= n && (ND == 2 || z <= n);
      if (!ok[u]) {
        x = 1;
        y = 1;
        z = ND == 3 ? 1 : 0;
      }
      const int64_t row = ND == 3 ? (int64_t)z * side + y : (int64_t)y;
      g[u] = gather(z, y, x);
      zo[u] = row * pz + x;
      yv[u] = HASY ? ldx(ys, row * py + x) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t v = E.template put<kVarGen>(g[u], yv[u], ok[u]);
      if (PASS != kQ1 && ok[u]) stv(zp, zbits, zo[u], v);
    }
  }
  ex_finish(E, ma.lm[ma.s[kOpZ]]);
}

template <int ND, int PASS, bool HASY>
__device__ __forceinline__ void ex_star(const StarLaunch& L, const OpArgs& op, const LdsMeta& ma) {
  const Src xs = src_of(L.x, L.xbits);
  const int n = (int)L.n;
  const int64_t px = L.px, side = L.n + 2, zs = side * L.px;
  int32_t t[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) t[k] = L.taps[k];
  ex_loop<ND, PASS, HASY, 4>(op, ma, n, L.y, L.ybits, L.py, L.z, L.zbits, L.pz,
                          [&](int z, int y, int x) -> int64_t {
    const int64_t b = (ND == 3 ? (int64_t)z * side + y : (int64_t)y) * px + x;
    int64_t g = (int64_t)t[0] * ldx(xs, b) + (int64_t)t[1] * ldx(xs, b - 1) +
                (int64_t)t[2] * ldx(xs, b + 1) + (int64_t)t[3] * ldx(xs, b - px) +
                (int64_t)t[4] * ldx(xs, b + px);
    if (ND == 3) g += (int64_t)t[5] * ldx(xs, b - zs) + (int64_t)t[6] * ldx(xs, b + zs);
    return g;
  });
}

template <int ND>
__device__ __forceinline__ constexpr int tidx(int iz, int iy, int ix) {
  return ND == 3 ? (iz * 3 + iy) * 3 + ix : iy * 3 + ix;
}

// restriction: z[I] = sum_o t[o] x[2I + o] over the 3^ND offsets
template <int ND, int PASS, bool HASY>
__device__ __forceinline__ void ex_restrict(const TransferLaunch& L, const OpArgs& op, const LdsMeta& ma) {
  const Src xs = src_of(L.x, L.xbits);
  const int64_t px = L.px, sf = L.n_in + 2;
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  ex_loop<ND, PASS, HASY, ND == 3 ? 1 : 2>(op, ma, (int)L.n_out, L.y, L.ybits, L.py, L.z,
                                           L.zbits, L.pz, [&](int z, int y, int x) -> int64_t {
    int64_t g = 0;
#pragma unroll
    for (int oz = (ND == 3 ? -1 : 0); oz <= (ND == 3 ? 1 : 0); ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy) {
        const int64_t row = ND == 3 ? (int64_t)(2 * z + oz) * sf + (2 * y + oy) : (int64_t)(2 * y + oy);
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox)
          g += (int64_t)t[tidx<ND>(oz + 1, oy + 1, ox + 1)] * ldx(xs, row * px + 2 * x + ox);
      }
    return g;
  });
}

// prolongation: fine node p takes t[2J - p] x[J] from the coarse nodes J
// with |2J - p| <= 1 per dimension: J = floor(p / 2) + e, e in {0,1}^ND,
// where along an even dimension only e = 0 contributes (offset 0) and along
// an odd one e selects the offset 2e - 1. The tap of each corner is chosen
// from the parities with selects, so the loads stay branch-free.
template <int ND, int PASS, bool HASY>
__device__ __forceinline__ void ex_prolong(const TransferLaunch& L, const OpArgs& op, const LdsMeta& ma) {
  const Src xs = src_of(L.x, L.xbits);
  const int64_t px = L.px, sc = L.n_in + 2;
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  ex_loop<ND, PASS, HASY, ND == 3 ? 1 : 2>(op, ma, (int)L.n_out, L.y, L.ybits, L.py, L.z,
                                           L.zbits, L.pz, [&](int z, int y, int x) -> int64_t {
    const int qz = z & 1, qy = y & 1, qx = x & 1;
    const int jz = z >> 1, jy = y >> 1, jx = x >> 1;
    int64_t g = 0;
#pragma unroll
    for (int ez = 0; ez < (ND == 3 ? 2 : 1); ++ez)
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
          int32_t tap = 0;
#pragma unroll
          for (int pz = 0; pz < (ND == 3 ? 2 : 1); ++pz)
#pragma unroll
            for (int py = 0; py < 2; ++py)
#pragma unroll
              for (int pxp = 0; pxp < 2; ++pxp) {
                const bool used = (ND == 2 || pz || !ez) && (py || !ey) && (pxp || !ex);
                const int iz = pz ? 2 * ez : 1, iy = py ? 2 * ey : 1, ix = pxp ? 2 * ex : 1;
                const int32_t cand = used ? t[tidx<ND>(iz, iy, ix)] : 0;
                const bool match = (ND == 2 || pz == qz) && py == qy && pxp == qx;
                tap = match ? cand : tap;
              }
          const int64_t row = ND == 3 ? (int64_t)(jz + ez) * sc + (jy + ey) : (int64_t)(jy + ey);
          g += (int64_t)tap * ldx(xs, row * px + jx + ex);
        }
    return g;
  });
}

template <int ND, int PASS, bool HASY>
__device__ __forceinline__ void ex_point(const PointLaunch& L, const OpArgs& op, const LdsMeta& ma) {
  const Src xs = src_of(L.x, L.xbits);
  const int64_t px = L.px, side = L.n + 2;
  ex_loop<ND, PASS, HASY, 4>(op, ma, (int)L.n, L.y, L.ybits, L.py, L.z, L.zbits, L.pz,
                          [&](int z, int y, int x) -> int64_t {
    const int64_t row = ND == 3 ? (int64_t)z * side + y : (int64_t)y;
    return ldx(xs, row * px + x);
  });
}

__device__ __forceinline__ void ex_zero(const ZeroOp& Z, int64_t* zm) {
  uint4* p = static_cast<uint4*>(Z.mant);
  const int64_t n16 = Z.bytes / 16;
  for (int64_t i = threadIdx.x; i < n16; i += kExecThreads) p[i] = make_uint4(0, 0, 0, 0);
  if (threadIdx.x < kExMetaF)
    zm[threadIdx.x] = threadIdx.x == kMetaExp ? Z.exp : (threadIdx.x == kMetaMu ? 1 : 0);
}

__device__ __forceinline__ OpArgs with_mode(const OpArgs& a, int mode) {
  OpArgs op = a;
  op.mode = mode;
  return op;
}

template <int ND, int PASS, bool HASY>
__device__ __forceinline__ void ex_dispatch(const ExecOp& op, MetaRow* lm, int mode) {
  const LdsMeta ma = lds_meta(lm, op.slot);
  if (op.kind == kExStar) {
    ex_star<ND, PASS, HASY>(op.u.star, with_mode(op.u.star.op, mode), ma);
  } else if (op.kind == kExPoint) {
    ex_point<ND, PASS, HASY>(op.u.pt, with_mode(op.u.pt.op, mode), ma);
  } else {
    const OpArgs a = with_mode(op.u.tr.op, mode);
    if (op.u.tr.kind == 1) ex_restrict<ND, PASS, HASY>(op.u.tr, a, ma);
    else ex_prolong<ND, PASS, HASY>(op.u.tr, a, ma);
  }
}

constexpr int kOpWords = (int)(sizeof(ExecOp) / 4);
static_assert(sizeof(ExecOp) % 4 == 0 && kOpWords <= kExecThreads, "ExecOp copy layout");

template <int ND>
__global__ __launch_bounds__(kExecThreads) void k_exec(const ExecOp* __restrict__ ops, int count,
                                                      int64_t* const* __restrict__ metas,
                                                      int nmeta) {
  __shared__ MetaRow lm[kExecMaxMeta];
  __shared__ ExecOp buf[2];
  const int t = threadIdx.x;
  const uint32_t* gw = reinterpret_cast<const uint32_t*>(ops);
  uint32_t* bw = reinterpret_cast<uint32_t*>(buf);
  if (t < nmeta * kExMetaF)
    lm[t / kExMetaF][t % kExMetaF] = ((const BFP_GLOBAL int64_t*)metas[t / kExMetaF])[t % kExMetaF];
  if (t < kOpWords) bw[t] = gw[t];
  __syncthreads();
  for (int k = 0; k < count; ++k) {
    // prefetch op k + 1 (its LDS copy is written once op k has finished)
    const bool pre = t < kOpWords && k + 1 < count;
    const uint32_t nextw = pre ? gw[(int64_t)(k + 1) * kOpWords + t] : 0;
    const ExecOp& op = buf[k & 1];
    if (op.kind == kExZero) {
      ex_zero(op.u.zero, lm[op.slot[2]]);
    } else {
      const int hasy = op.kind == kExStar ? op.u.star.op.has_y
                                          : (op.kind == kExPoint ? op.u.pt.op.has_y
                                                                 : op.u.tr.op.has_y);
      if (op.mode == kExModeQ) {
        if (hasy) {
          ex_dispatch<ND, kQ1, true>(op, lm, kModeQ1);
          ex_dispatch<ND, kOut, true>(op, lm, kModeQ2);
        } else {
          ex_dispatch<ND, kQ1, false>(op, lm, kModeQ1);
          ex_dispatch<ND, kOut, false>(op, lm, kModeQ2);
        }
      } else if (hasy) {
        ex_dispatch<ND, kOut, true>(op, lm, op.mode);
      } else {
        ex_dispatch<ND, kOut, false>(op, lm, op.mode);
      }
    }
    if (pre) bw[((k + 1) & 1) * kOpWords + t] = nextw;
    __syncthreads();
  }
  if (t < nmeta * kExMetaF)
    ((BFP_GLOBAL int64_t*)metas[t / kExMetaF])[t % kExMetaF] = lm[t / kExMetaF][t % kExMetaF];
}

}  // namespace

hipError_t launch_exec(const ExecOp* ops_dev, int count, int64_t* const* metas_dev, int nmeta,
                       int ndim, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (nmeta < 1 || nmeta > kExecMaxMeta) return hipErrorInvalidValue;
  if (ndim == 2)
    hipLaunchKernelGGL(k_exec<2>, dim3(1), dim3(kExecThreads), 0, s, ops_dev, count, metas_dev, nmeta);
  else
    hipLaunchKernelGGL(k_exec<3>, dim3(1), dim3(kExecThreads), 0, s, ops_dev, count, metas_dev, nmeta);
  return hipGetLastError();
}

}  // namespace bfpk
