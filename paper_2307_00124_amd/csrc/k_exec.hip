// Coarse-level executor: one workgroup runs a recorded list of BFP
// operations (star stencils, grid transfers, pointwise ops, zero fills,
// FP64 conversions) one after the other, with a workgroup barrier between
// them. Each operation computes exactly what its stand-alone kernel computes
// — the same exact row sums and the same epilogue (the generic exact
// combine) — and publishes its metadata from a workgroup reduction, so a
// whole coarse V-cycle, or the coarse levels of FMG, cost one launch instead
// of one or two launches per operation. The batched form runs one such
// workgroup per independent problem: a whole FMG solve per workgroup, every
// problem of a batch in one launch.
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
//
// Programs of batched problems are relocatable: their data and metadata
// pointers are offsets that the executor adds to the problem's arena base
// (base 0 for the absolute programs of a single hierarchy).
#include "epilogue.hpp"

namespace bfpk {

namespace {

// Pointers read from the recorded ops are generic; the data all lives in
// global memory, and saying so keeps loads and stores off the flat path
// (whose waits would also cover the LDS traffic of the executor).
#define BFP_GLOBAL __attribute__((address_space(1)))

struct Src {
  const BFP_GLOBAL char* p;
  int sh;     // log2 of the element size in bytes
  int bits;
};

// relocation of a recorded pointer by the running problem's base
__device__ __forceinline__ void* rel(const void* p, uintptr_t base) {
  return (void*)((uintptr_t)p + base);
}

__device__ __forceinline__ Src src_of(const void* p, int bits, uintptr_t base) {
  return Src{(const BFP_GLOBAL char*)rel(p, base), bits == 32 ? 2 : (bits == 16 ? 1 : 0), bits};
}

// element i, sign-extended from its storage width (W32: every operand of
// the op is stored in 32 bits, a plain load)
template <bool W32>
__device__ __forceinline__ int32_t ldx(const Src& s, int64_t i) {
  if (W32) return ((const BFP_GLOBAL int32_t*)s.p)[i];
  const int64_t off = i << s.sh;
  const uint32_t word = *(const BFP_GLOBAL uint32_t*)(s.p + (off & ~(int64_t)3));
  const int at = (int)(off & 3) * 8;
  return (int32_t)(word << (32 - s.bits - at)) >> (32 - s.bits);
}

template <bool W32>
__device__ __forceinline__ void stv(void* p, int bits, int64_t i, int64_t v) {
  if (W32 || bits == 32) ((BFP_GLOBAL int32_t*)p)[i] = (int32_t)v;
  else if (bits == 16) ((BFP_GLOBAL int16_t*)p)[i] = (int16_t)v;
  else ((BFP_GLOBAL int8_t*)p)[i] = (int8_t)v;
}

typedef int64_t MetaRow[kExMetaF];

// What an op leaves to publish once the program loop's barrier has passed:
// the workgroup reduction of its outputs (every wave reduces the per-wave
// partials itself and writes the same metadata into the LDS mirror, so no
// wave waits for another's serial tail), or a zero fill's metadata. Kept
// in registers, uniformly, by every wave.
constexpr int kFinNone = 0, kFinOut = 1, kFinZero = 2;
struct Fin {
  MetaRow* z;
  int kind;
  int par;          // which half of the double-buffered partials
  int64_t eo;       // output exponent
  int64_t* diag;    // diagnostics of the op (DG programs only)
  int dbin, dsat;
};

// Operand metadata read from the LDS mirror by slot.
struct PendingDiag;
struct LdsMeta {
  MetaRow* lm;
  PendingDiag* pend;   // where the op leaves its diagnostic counts
  Fin* fin;            // the op's pending publication
  int32_t* red;        // per-wave partials: [2][3][waves] outputs, then [waves] mu
  int s[5];
  __device__ __forceinline__ int64_t operator()(int k, int f) const { return lm[s[k]][f]; }
};

__device__ __forceinline__ LdsMeta lds_meta(MetaRow* lm, PendingDiag* pend, Fin* fin,
                                            int32_t* red, const int16_t* slot) {
  LdsMeta m;
  m.lm = lm;
  m.pend = pend;
  m.fin = fin;
  m.red = red;
  m.s[kOpX] = slot[0];
  m.s[kOpY] = slot[1] >= 0 ? slot[1] : slot[0];
  m.s[kOpZ] = slot[2];
  m.s[kOpGa] = slot[3] >= 0 ? slot[3] : 0;
  m.s[kOpGb] = slot[4] >= 0 ? slot[4] : 0;
  return m;
}

// After one lane (or a few) of a wave wrote metadata rows that every lane
// reads next: the wave's LDS accesses execute in order, so only the
// compiler must be kept from moving the other lanes' reads above the
// writes (which it may do without a fence: no write is on their path).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// An op's diagnostic counts, left by its reduction for thread 0 to issue
// at the start of the next op (then nothing on the op's own path waits for
// the atomics' acknowledgement).
struct PendingDiag {
  int64_t* diag;
  int dbin, dsat;
  int64_t nsat;
};

// Workgroup reductions: per-wave partials (DPP) in LDS.
// Single-hierarchy programs (latency-bound: one workgroup on the GPU) let
// every wave reduce the partials itself: the first qcomp pass needs mu* at
// once (one barrier, then each wave writes the same mu* into the output's
// row); an output pass only leaves its partials, published after the
// program loop's barrier (the one that also makes the op's stores
// visible), so an op costs one barrier per pass and no wave waits behind a
// serial tail. Batched programs (many workgroups per CU: throughput-bound)
// keep the cheaper form: wave 0 alone reduces after a barrier and writes
// the row before the next barrier.
template <int NT>
constexpr bool ex_latency_form() {
  return NT > kBatchThreads;
}

template <int NT, int PASS, bool HASY, bool DG>
__device__ __forceinline__ void ex_finish(const Epi<PASS, HASY, DG>& E, const LdsMeta& ma) {
  constexpr int kW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  MetaRow& zm = ma.lm[ma.s[kOpZ]];
  if (PASS == kQ1) {
    int32_t* r = ma.red + 6 * kW;
    const int32_t m = wave_max32((int32_t)E.tmu);
    if (lane == 0) r[wave] = m;
    __syncthreads();
    if constexpr (ex_latency_form<NT>()) {
      int32_t b = 1;
#pragma unroll
      for (int k = 0; k < kW; ++k) b = r[k] > b ? r[k] : b;
      if (lane == 0) zm[kMetaMu] = b;
      wave_sync_lds();
    } else {
      if (wave == 0) {
        const int32_t b = wave_max32(lane < kW ? r[lane] : 1);
        if (lane == 0) zm[kMetaMu] = b;
      }
      __syncthreads();   // the second pass reads mu* at once
    }
  } else {
    Fin& f = *ma.fin;
    int32_t* r = ma.red + f.par * 3 * kW;
    const int32_t a = wave_max32(E.tmax), b = wave_min32(E.tmin), c = wave_sum32(E.tsat);
    if (lane == 0) {
      r[wave] = a;
      r[kW + wave] = b;
      r[2 * kW + wave] = c;
    }
    if constexpr (ex_latency_form<NT>()) {
      f.z = &zm;
      f.kind = kFinOut;
      f.eo = E.R.eo;
      f.diag = DG ? E.diag : nullptr;
      f.dbin = E.dbin;
      f.dsat = E.dsat;
    } else {
      __syncthreads();
      if (wave == 0) {
        const bool in = lane < kW;
        const int32_t mx = wave_max32(in ? r[lane] : 0);
        const int32_t mn = wave_min32(in ? r[kW + lane] : 0);
        const int32_t st = wave_sum32(in ? r[2 * kW + lane] : 0);
        if (lane == 0) {
          zm[kMetaMax] = mx;
          zm[kMetaMin] = mn;
          zm[kMetaSat] = st;
          zm[kMetaExp] = E.R.eo;
          if (DG && E.diag) *ma.pend = PendingDiag{E.diag, E.dbin, E.dsat, st};
        }
      }
      // the program loop's barrier follows before any reader
    }
  }
}

// Publish the previous op's metadata (after the program loop's barrier;
// latency form only).
template <int NT, bool DG>
__device__ __forceinline__ void ex_publish(Fin& f, const int32_t* red, PendingDiag& pend) {
  constexpr int kW = NT / 64;
  const int lane = threadIdx.x & 63;
  if (f.kind == kFinNone) return;
  if (f.kind == kFinOut) {
    const int32_t* r = red + f.par * 3 * kW;
    int32_t mx = 0, mn = 0, st = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      mx = r[k] > mx ? r[k] : mx;
      mn = r[kW + k] < mn ? r[kW + k] : mn;
      st += r[2 * kW + k];
    }
    if (lane == 0) {
      (*f.z)[kMetaMax] = mx;
      (*f.z)[kMetaMin] = mn;
      (*f.z)[kMetaSat] = st;
      (*f.z)[kMetaExp] = f.eo;
    }
    if (DG && threadIdx.x == 0 && f.diag) pend = PendingDiag{f.diag, f.dbin, f.dsat, st};
  } else if (f.kind == kFinZero) {
    if (lane < kExMetaF) (*f.z)[lane] = lane == kMetaExp ? f.eo : (lane == kMetaMu ? 1 : 0);
  }
  wave_sync_lds();
  f.kind = kFinNone;
}

// Visit every interior point (z, y, x) of an n^ND output grid: the exact
// value g = gather(z, y, x), the optional y entry, the epilogue and the store.
// Points are enumerated on a 2^lg >= n padded index space; a padding slot
// becomes the interior point (1, 1, 1), which keeps every address in bounds,
// and is neither stored nor counted.
__device__ __forceinline__ OpArgs with_mode(const OpArgs& a, int mode) {
  OpArgs op = a;
  op.mode = mode;
  return op;
}

// PASS = kQF: both qcomp passes of one op. When every output point fits
// one round (U points per thread) the exact values are gathered once, kept
// in registers across the mu* reduction and quantized from there (the same
// values the second pass would gather again: the first stores nothing);
// otherwise the two passes run one after the other.
constexpr int kQF = 3;

template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32, int U, typename Gather>
__device__ __forceinline__ void ex_loop(const OpArgs& op, const LdsMeta& ma, uintptr_t base,
                                        int n, const void* yp, int ybits, int64_t py, void* zp0,
                                        int zbits, int64_t pz, Gather&& gather) {
  if constexpr (PASS == kQF) {
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const int tot = ND == 3 ? 1 << (3 * lg) : 1 << (2 * lg);
    const OpArgs q1 = with_mode(op, kModeQ1), q2 = with_mode(op, kModeQ2);
    if (tot > U * NT) {
      ex_loop<NT, ND, kQ1, HASY, DG, W32, U>(q1, ma, base, n, yp, ybits, py, zp0, zbits, pz, gather);
      ex_loop<NT, ND, kOut, HASY, DG, W32, U>(q2, ma, base, n, yp, ybits, py, zp0, zbits, pz, gather);
      return;
    }
    const int M = (1 << lg) - 1;
    const int64_t side = n + 2;
    const Src ys = src_of(yp, ybits, base);
    void* zp = rel(zp0, base);
    Epi<kQ1, HASY, DG> E1;
    E1.init(q1, ma);
    int64_t g[U], zo[U];
    int32_t yv[U];
    bool ok[U];
    // rounds holding a point of this wave (the rest are skipped uniformly;
    // latency form only: in batched programs every round keeps its loads
    // in one straight run)
    const int w0 = ex_latency_form<NT>() ? __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63 : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = false;
      g[u] = 0;
      zo[u] = 0;
      yv[u] = 0;
      if (ex_latency_form<NT>() && w0 + u * NT >= tot) continue;
      const int i = threadIdx.x + u * NT;
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
      yv[u] = HASY ? ldx<W32>(ys, row * py + x) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (!ex_latency_form<NT>() || w0 + u * NT < tot) E1.template put<kVarGen>(g[u], yv[u], ok[u]);
    ex_finish<NT>(E1, ma);   // mu*, after one barrier
    Epi<kOut, HASY, DG> E2;
    E2.init(q2, ma);
    auto store = [&](auto var_tag) {
      constexpr int VAR = decltype(var_tag)::value;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ex_latency_form<NT>() && w0 + u * NT >= tot) continue;
        const int64_t v = E2.template put<VAR>(g[u], yv[u], ok[u]);
        if (ok[u]) stv<W32>(zp, zbits, zo[u], v);
      }
    };
    if (E2.fast) store(std::integral_constant<int, kVarFast>());
    else store(std::integral_constant<int, kVarGen>());
    ex_finish<NT>(E2, ma);
    return;
  } else {
  Epi<PASS, HASY, DG> E;
  E.init(op, ma);
  const Src ys = src_of(yp, ybits, base);
  void* zp = rel(zp0, base);
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const int M = (1 << lg) - 1;
  const int tot = ND == 3 ? 1 << (3 * lg) : 1 << (2 * lg);
  const int64_t side = n + 2;
  auto body = [&](auto var_tag) {
    constexpr int VAR = decltype(var_tag)::value;
    const int w0 = ex_latency_form<NT>() ? __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63 : 0;
    for (int r0 = 0; (ex_latency_form<NT>() ? w0 : (int)threadIdx.x) + r0 < tot; r0 += U * NT) {
      const int i0 = threadIdx.x + r0;
      int64_t g[U], zo[U];
      int32_t yv[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ok[u] = false;
        g[u] = 0;
        zo[u] = 0;
        yv[u] = 0;
        if (ex_latency_form<NT>() && w0 + r0 + u * NT >= tot) continue;
        const int i = i0 + u * NT;
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
        yv[u] = HASY ? ldx<W32>(ys, row * py + x) : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ex_latency_form<NT>() && w0 + r0 + u * NT >= tot) continue;
        const int64_t v = E.template put<VAR>(g[u], yv[u], ok[u]);
        if (PASS != kQ1 && ok[u]) stv<W32>(zp, zbits, zo[u], v);
      }
    }
  };
  // the fast epilogue when no intermediate can overflow (decided once per op)
  if (PASS != kQ1 && E.fast) body(std::integral_constant<int, kVarFast>());
  else body(std::integral_constant<int, kVarGen>());
  ex_finish<NT>(E, ma);
  }
}

// Points per thread and round of the star and pointwise ops: four in 2D;
// in 3D (grids of at most 15^3 here) two in the single-hierarchy executor
// and one in the batched one and in the programs that count diagnostics,
// which keeps the 3D op code within the register file (more in flight
// spilled to scratch).
template <int NT, int ND, bool DG>
constexpr int ex_rounds() {
  return ND == 2 ? 4 : (NT > kBatchThreads && !DG ? 2 : 1);
}

template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32>
__device__ __forceinline__ void ex_star(const StarLaunch& L, const OpArgs& op, const LdsMeta& ma,
                                     uintptr_t base) {
  const Src xs = src_of(L.x, L.xbits, base);
  const int n = (int)L.n;
  const int64_t px = L.px, side = L.n + 2, zs = side * L.px;
  int32_t t[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) t[k] = L.taps[k];
  ex_loop<NT, ND, PASS, HASY, DG, W32, ex_rounds<NT, ND, DG>()>(op, ma, base, n, L.y, L.ybits, L.py, L.z, L.zbits, L.pz,
                          [&](int z, int y, int x) -> int64_t {
    const int64_t b = (ND == 3 ? (int64_t)z * side + y : (int64_t)y) * px + x;
    int64_t g = (int64_t)t[0] * ldx<W32>(xs, b) + (int64_t)t[1] * ldx<W32>(xs, b - 1) +
                (int64_t)t[2] * ldx<W32>(xs, b + 1) + (int64_t)t[3] * ldx<W32>(xs, b - px) +
                (int64_t)t[4] * ldx<W32>(xs, b + px);
    if (ND == 3) g += (int64_t)t[5] * ldx<W32>(xs, b - zs) + (int64_t)t[6] * ldx<W32>(xs, b + zs);
    return g;
  });
}

template <int ND>
__device__ __forceinline__ constexpr int tidx(int iz, int iy, int ix) {
  return ND == 3 ? (iz * 3 + iy) * 3 + ix : iy * 3 + ix;
}

// restriction: z[I] = sum_o t[o] x[2I + o] over the 3^ND offsets
template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32>
__device__ __forceinline__ void ex_restrict(const TransferLaunch& L, const OpArgs& op, const LdsMeta& ma,
                                     uintptr_t base) {
  const Src xs = src_of(L.x, L.xbits, base);
  const int64_t px = L.px, sf = L.n_in + 2;
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  ex_loop<NT, ND, PASS, HASY, DG, W32, ND == 3 ? 1 : 2>(op, ma, base, (int)L.n_out, L.y, L.ybits,
                                               L.py, L.z, L.zbits, L.pz, [&](int z, int y, int x) -> int64_t {
    int64_t g = 0;
#pragma unroll
    for (int oz = (ND == 3 ? -1 : 0); oz <= (ND == 3 ? 1 : 0); ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy) {
        const int64_t row = ND == 3 ? (int64_t)(2 * z + oz) * sf + (2 * y + oy) : (int64_t)(2 * y + oy);
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox)
          g += (int64_t)t[tidx<ND>(oz + 1, oy + 1, ox + 1)] * ldx<W32>(xs, row * px + 2 * x + ox);
      }
    return g;
  });
}

// prolongation: fine node p takes t[2J - p] x[J] from the coarse nodes J
// with |2J - p| <= 1 per dimension: J = floor(p / 2) + e, e in {0,1}^ND,
// where along an even dimension only e = 0 contributes (offset 0) and along
// an odd one e selects the offset 2e - 1. The tap of each corner is chosen
// from the parities with selects, so the loads stay branch-free.
template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32>
__device__ __forceinline__ void ex_prolong(const TransferLaunch& L, const OpArgs& op, const LdsMeta& ma,
                                     uintptr_t base) {
  const Src xs = src_of(L.x, L.xbits, base);
  const int64_t px = L.px, sc = L.n_in + 2;
  int32_t t[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) t[k] = L.taps[k];
  ex_loop<NT, ND, PASS, HASY, DG, W32, ND == 3 ? 1 : 2>(op, ma, base, (int)L.n_out, L.y, L.ybits,
                                               L.py, L.z, L.zbits, L.pz, [&](int z, int y, int x) -> int64_t {
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
          g += (int64_t)tap * ldx<W32>(xs, row * px + jx + ex);
        }
    return g;
  });
}

template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32>
__device__ __forceinline__ void ex_point(const PointLaunch& L, const OpArgs& op, const LdsMeta& ma,
                                     uintptr_t base) {
  const Src xs = src_of(L.x, L.xbits, base);
  const int64_t px = L.px, side = L.n + 2;
  ex_loop<NT, ND, PASS, HASY, DG, W32, ex_rounds<NT, ND, DG>()>(op, ma, base, (int)L.n, L.y, L.ybits, L.py, L.z, L.zbits, L.pz,
                          [&](int z, int y, int x) -> int64_t {
    const int64_t row = ND == 3 ? (int64_t)z * side + y : (int64_t)y;
    return ldx<W32>(xs, row * px + x);
  });
}

// (latency form: the metadata is published after the loop's barrier, like
// an op's)
template <int NT>
__device__ __forceinline__ void ex_zero(const ZeroOp& Z, MetaRow* zm, Fin& fin, uintptr_t base) {
  uint4* p = static_cast<uint4*>(rel(Z.mant, base));
  const int64_t n16 = Z.bytes / 16;
  for (int64_t i = threadIdx.x; i < n16; i += NT) p[i] = make_uint4(0, 0, 0, 0);
  if constexpr (ex_latency_form<NT>()) {
    fin.z = zm;
    fin.kind = kFinZero;
    fin.eo = Z.exp;
  } else if (threadIdx.x < kExMetaF) {
    (*zm)[threadIdx.x] = threadIdx.x == kMetaExp ? Z.exp : (threadIdx.x == kMetaMu ? 1 : 0);
  }
}


template <int NT, int ND, int PASS, bool HASY, bool DG, bool W32>
__device__ __forceinline__ void ex_dispatch(const ExecOp& op, MetaRow* lm, PendingDiag* pend,
                                            Fin* fin, int32_t* red, int mode, uintptr_t base) {
  const LdsMeta ma = lds_meta(lm, pend, fin, red, op.slot);
  if (op.kind == kExStar) {
    ex_star<NT, ND, PASS, HASY, DG, W32>(op.u.star, with_mode(op.u.star.op, mode), ma, base);
  } else if (op.kind == kExPoint) {
    ex_point<NT, ND, PASS, HASY, DG, W32>(op.u.pt, with_mode(op.u.pt.op, mode), ma, base);
  } else {
    const OpArgs a = with_mode(op.u.tr.op, mode);
    if (op.u.tr.kind == 1) ex_restrict<NT, ND, PASS, HASY, DG, W32>(op.u.tr, a, ma, base);
    else ex_prolong<NT, ND, PASS, HASY, DG, W32>(op.u.tr, a, ma, base);
  }
}

// FP64 -> BFP (normalized floor quantization, the bfp_vec_from_f64
// result): the largest nu(x_i) over the interior, then
// m_i = floor(x_i / 2^(max nu - w)), exponent max nu - w + log2_scale.
__device__ __forceinline__ bool f64_split(double x, int64_t& z, int64_t& e, bool& finite) {
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

template <int NT, int ND>
__device__ __forceinline__ void ex_conv(const ConvOp& C, MetaRow& zm, uintptr_t base,
                                        const double* const* rhs) {
  __shared__ int32_t cred[3][NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const BFP_GLOBAL double* src =
      (const BFP_GLOBAL double*)(C.src ? (const void*)C.src : (const void*)rhs[C.level - 1]);
  const int n = (int)C.n;
  const int64_t side = C.n + 2;
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const int M = (1 << lg) - 1;
  const int tot = ND == 3 ? 1 << (3 * lg) : 1 << (2 * lg);
  // pass 1: max nu and the non-finite flag
  int32_t best = INT32_MIN, bad = 0;
  for (int i = t; i < tot; i += NT) {
    const int x = (i & M) + 1, y = ((i >> lg) & M) + 1, z = ND == 3 ? (i >> (2 * lg)) + 1 : 0;
    if (x > n || y > n || (ND == 3 && z > n)) continue;
    const int64_t idx = (ND == 3 ? (int64_t)z * side + y : (int64_t)y) * side + x;
    int64_t zz, e;
    bool fin;
    if (f64_split(src[idx], zz, e, fin)) {
      const int32_t nu = (int32_t)(msb64(zz) + e);
      best = nu > best ? nu : best;
    }
    bad |= !fin;
  }
  best = wave_max32(best);
  bad = wave_max32(bad);
  if (lane == 0) {
    cred[0][wave] = best;
    cred[1][wave] = bad;
  }
  __syncthreads();
  int32_t numax = INT32_MIN, anybad = 0;
  for (int k = 0; k < NT / 64; ++k) {
    numax = cred[0][k] > numax ? cred[0][k] : numax;
    anybad |= cred[1][k];
  }
  const int64_t eq = numax == INT32_MIN ? 1 - C.w : (int64_t)numax - C.w;
  // pass 2: quantize and store
  void* mant = rel(C.mant, base);
  int32_t tmax = 0, tmin = 0;
  for (int i = t; i < tot; i += NT) {
    const int x = (i & M) + 1, y = ((i >> lg) & M) + 1, z = ND == 3 ? (i >> (2 * lg)) + 1 : 0;
    if (x > n || y > n || (ND == 3 && z > n)) continue;
    const int64_t row = ND == 3 ? (int64_t)z * side + y : (int64_t)y;
    int64_t zz, e, v = 0;
    bool fin;
    if (f64_split(src[row * side + x], zz, e, fin)) {
      const int64_t sh = e - eq;
      v = sh >= 0 ? (int64_t)((uint64_t)zz << sh) : shr_floor(zz, -sh);
    }
    tmax = (int32_t)v > tmax ? (int32_t)v : tmax;
    tmin = (int32_t)v < tmin ? (int32_t)v : tmin;
    stv<false>(mant, C.bits, row * C.pitch + x, v);
  }
  tmax = wave_max32(tmax);
  tmin = wave_min32(tmin);
  __syncthreads();   // cred is reused
  if (lane == 0) {
    cred[0][wave] = tmax;
    cred[1][wave] = tmin;
  }
  __syncthreads();
  if (t == 0) {
    int32_t mx = 0, mn = 0;
    for (int k = 0; k < NT / 64; ++k) {
      mx = cred[0][k] > mx ? cred[0][k] : mx;
      mn = cred[1][k] < mn ? cred[1][k] : mn;
    }
    zm[kMetaExp] = eq + C.log2_scale;
    zm[kMetaMax] = mx;
    zm[kMetaMin] = mn;
    zm[kMetaSat] = 0;
    zm[kMetaMu] = numax == INT32_MIN ? INT64_MIN : (int64_t)numax;
    zm[kMetaFlags] |= anybad;
  }
}

constexpr int kOpWords = (int)(sizeof(ExecOp) / 4);
static_assert(sizeof(ExecOp) % 4 == 0 && kOpWords <= kBatchThreads, "ExecOp copy layout");

// Run one program (ops[0..count), metadata table metas[0..nmeta)) with this
// workgroup; pointers are relocated by `base`. SPEC32: ops whose operands
// are all stored in 32 bits take plain loads and stores (a second copy of
// the op code, kept to the single-hierarchy programs without diagnostics).
template <int NT, int ND, bool DG, bool SPEC32>
__device__ __forceinline__ void run_program(const ExecOp* __restrict__ ops, int count,
                                            int64_t* const* __restrict__ metas, int nmeta,
                                            uintptr_t base, const double* const* rhs) {
  __shared__ MetaRow lm[kExecMaxMeta];
  __shared__ ExecOp buf[2];
  __shared__ PendingDiag pend;
  __shared__ int32_t red[7 * (NT / 64)];
  Fin fin;
  fin.kind = kFinNone;
  fin.par = 0;
  const int t = threadIdx.x;
  if (DG && t == 0) pend.diag = nullptr;
  const uint32_t* gw = reinterpret_cast<const uint32_t*>(ops);
  uint32_t* bw = reinterpret_cast<uint32_t*>(buf);
  for (int i = t; i < nmeta * kExMetaF; i += NT)
    lm[i / kExMetaF][i % kExMetaF] = ((const BFP_GLOBAL int64_t*)rel(metas[i / kExMetaF], base))[i % kExMetaF];
  if (t < kOpWords) bw[t] = gw[t];
  __syncthreads();
  for (int k = 0; k < count; ++k) {
    // prefetch op k + 1 (its LDS copy is written once op k has finished)
    const bool pre = t < kOpWords && k + 1 < count;
    const uint32_t nextw = pre ? gw[(int64_t)(k + 1) * kOpWords + t] : 0;
    const ExecOp& op = buf[k & 1];
    if (DG && t == 0 && pend.diag) {   // the previous op's diagnostic counts
      diag_count(pend.diag, pend.dbin, pend.dsat, pend.nsat);
      pend.diag = nullptr;
    }
    fin.par = k & 1;
    if (op.kind == kExZero) {
      ex_zero<NT>(op.u.zero, &lm[op.slot[2]], fin, base);
    } else if (op.kind == kExConv) {
      ex_conv<NT, ND>(op.u.conv, lm[op.slot[2]], base, rhs);
    } else {
      const int hasy = op.kind == kExStar ? op.u.star.op.has_y
                                          : (op.kind == kExPoint ? op.u.pt.op.has_y
                                                                 : op.u.tr.op.has_y);
      auto run_op = [&](auto w32_tag) {
        constexpr bool W32 = decltype(w32_tag)::value;
        if (op.mode == kExModeQ) {
          if (hasy) ex_dispatch<NT, ND, kQF, true, DG, W32>(op, lm, &pend, &fin, red, kModeQ2, base);
          else ex_dispatch<NT, ND, kQF, false, DG, W32>(op, lm, &pend, &fin, red, kModeQ2, base);
        } else if (hasy) {
          ex_dispatch<NT, ND, kOut, true, DG, W32>(op, lm, &pend, &fin, red, op.mode, base);
        } else {
          ex_dispatch<NT, ND, kOut, false, DG, W32>(op, lm, &pend, &fin, red, op.mode, base);
        }
      };
      if constexpr (SPEC32) {
        int xb, yb, zb;
        if (op.kind == kExStar) {
          xb = op.u.star.xbits; yb = op.u.star.ybits; zb = op.u.star.zbits;
        } else if (op.kind == kExPoint) {
          xb = op.u.pt.xbits; yb = op.u.pt.ybits; zb = op.u.pt.zbits;
        } else {
          xb = op.u.tr.xbits; yb = op.u.tr.ybits; zb = op.u.tr.zbits;
        }
        if (xb == 32 && zb == 32 && (!hasy || yb == 32)) run_op(std::true_type());
        else run_op(std::false_type());
      } else {
        run_op(std::false_type());
      }
    }
    if (pre) bw[((k + 1) & 1) * kOpWords + t] = nextw;
    __syncthreads();
    ex_publish<NT, DG>(fin, red, pend);
  }
  __syncthreads();
  for (int i = t; i < nmeta * kExMetaF; i += NT)
    ((BFP_GLOBAL int64_t*)rel(metas[i / kExMetaF], base))[i % kExMetaF] = lm[i / kExMetaF][i % kExMetaF];
  if (DG && t == 0 && pend.diag) diag_count(pend.diag, pend.dbin, pend.dsat, pend.nsat);
}

// DG: the program counts diagnostics (otherwise their code is compiled out).
// One workgroup per launch: two waves per SIMD is all the occupancy there
// is, so the compiler may use the whole register file (no spills). The
// plain 32-bit op copy only in 2D (3D programs cover grids of at most 15^3).
template <int ND, bool DG>
__global__ __launch_bounds__(kExecThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_exec(const ExecOp* __restrict__ ops, int count,
                                                      int64_t* const* __restrict__ metas,
                                                      int nmeta, ExecRhs rhs) {
  // the right-hand-side pointers, for the program's conversions (read after
  // the program runner's first barrier)
  __shared__ const double* srhs[kMaxLevels];
  if (threadIdx.x < kMaxLevels) srhs[threadIdx.x] = rhs.p[threadIdx.x];
  run_program<kExecThreads, ND, DG, ND == 2 && !DG>(ops, count, metas, nmeta, 0, srhs);
}

template <int ND>
__global__ __launch_bounds__(kBatchThreads) void k_exec_batch(
    const BatchEntry* __restrict__ entries, const ExecOp* __restrict__ ops,
    int64_t* const* __restrict__ metas, const double* const* __restrict__ rhs_table) {
  const BatchEntry& E = entries[blockIdx.x];
  run_program<kBatchThreads, ND, false, false>(ops + E.op_begin, E.op_count, metas + E.meta_begin,
                                        E.nmeta, E.base, rhs_table + (int64_t)E.prob * kMaxLevels);
}

}  // namespace

hipError_t launch_exec_batch(const BatchEntry* entries_dev, int nentries, const ExecOp* ops_dev,
                             int64_t* const* metas_dev, const double* const* rhs_table_dev,
                             int ndim, hipStream_t s) {
  if (nentries <= 0) return hipSuccess;
  if (ndim == 2)
    hipLaunchKernelGGL(k_exec_batch<2>, dim3(nentries), dim3(kBatchThreads), 0, s, entries_dev,
                       ops_dev, metas_dev, rhs_table_dev);
  else
    hipLaunchKernelGGL(k_exec_batch<3>, dim3(nentries), dim3(kBatchThreads), 0, s, entries_dev,
                       ops_dev, metas_dev, rhs_table_dev);
  return hipGetLastError();
}

hipError_t launch_exec(const ExecOp* ops_dev, int count, int64_t* const* metas_dev, int nmeta,
                       int ndim, const ExecRhs* rhs, bool diag, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (nmeta < 1 || nmeta > kExecMaxMeta) return hipErrorInvalidValue;
  ExecRhs r{};
  if (rhs) r = *rhs;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(1), dim3(kExecThreads), 0, s, ops_dev, count, metas_dev, nmeta, r);
  };
  if (ndim == 2) diag ? go(k_exec<2, true>) : go(k_exec<2, false>);
  else diag ? go(k_exec<3, true>) : go(k_exec<3, false>);
  return hipGetLastError();
}

}  // namespace bfpk
