// Device-side integer primitives shared by every BFP kernel.
//
// Semantics (paper Section 2): two's-complement integers, arithmetic right
// shifts that round toward minus infinity, msb(v) = the smallest b >= 1 with
// v in X_b = [-2^(b-1), 2^(b-1) - 1] (so msb(0) = msb(-1) = 1, msb(23) = 6).
// Every routine here is exact; values that cannot fit the 62-bit budget are
// reported as +-2^62, which lies outside every representable output range
// (w_out <= 32), so a following clamp saturates them correctly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace bfpk {

constexpr int64_t kSatBig = (int64_t)1 << 62;

__device__ __forceinline__ int bitlen64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

__device__ __forceinline__ int msb64(int64_t v) {
  return bitlen64((uint64_t)(v ^ (v >> 63))) + 1;
}

__device__ __forceinline__ int msb128(__int128 v) {
  unsigned __int128 u = (unsigned __int128)(v ^ (v >> 127));
  uint64_t hi = (uint64_t)(u >> 64);
  return hi ? 64 + bitlen64(hi) + 1 : bitlen64((uint64_t)u) + 1;
}

// floor(v / 2^k) for k >= 0 (k may exceed 63).
__device__ __forceinline__ int64_t shr_floor(int64_t v, int64_t k) {
  return v >> (k > 63 ? 63 : (int)k);
}

// a * 2^k + c for k >= 0 with |a|, |c| < 2^61: exact when |a| 2^k < 2^62,
// otherwise +-2^62 with the sign of a (|a 2^k + c| then exceeds 2^61).
__device__ __forceinline__ int64_t shl_add_sat(int64_t a, int64_t k, int64_t c) {
  if (a == 0) return c;
  uint64_t mag = (uint64_t)(a < 0 ? -a : a);
  if (k + bitlen64(mag) >= 63) return a > 0 ? kSatBig : -kSatBig;
  return (int64_t)((uint64_t)a << k) + c;
}

// How floor(a 2^sa + b 2^sb) is evaluated without overflow. The term with
// the larger shift is "hi"; D = s_hi - s_lo >= 0.
//   kInt:       s_lo >= 0          value = (hi 2^D + lo) 2^s_lo
//   kHighShift: s_lo < 0, D >= L   value = hi 2^(D-L) + floor(lo / 2^L)
//   kShiftDown: s_lo < 0, D < L    value = floor((hi + floor(lo/2^D)) / 2^(L-D))
// with L = -s_lo (the last form is exact because hi is an integer).
enum { kInt = 0, kHighShift = 1, kShiftDown = 2 };

struct Combine {
  int kind;
  int swap;      // 1: hi is the second operand
  int64_t D, L, s_lo;
};

__device__ __forceinline__ Combine make_combine(int64_t sa, int64_t sb) {
  Combine c;
  c.swap = sa < sb;
  int64_t s_hi = c.swap ? sb : sa;
  int64_t s_lo = c.swap ? sa : sb;
  c.D = s_hi - s_lo;
  c.s_lo = s_lo;
  c.L = -s_lo;
  if (s_lo >= 0) c.kind = kInt;
  else if (c.D >= c.L) c.kind = kHighShift;
  else c.kind = kShiftDown;
  return c;
}

// floor(a 2^sa + b 2^sb), +-2^62 when beyond range. |a|, |b| < 2^61.
__device__ __forceinline__ int64_t combine(const Combine& c, int64_t a, int64_t b) {
  int64_t hi = c.swap ? b : a;
  int64_t lo = c.swap ? a : b;
  if (c.kind == kInt) {
    int64_t v = shl_add_sat(hi, c.D, lo);
    return c.s_lo == 0 ? v : shl_add_sat(v, c.s_lo, 0);
  }
  if (c.kind == kHighShift) return shl_add_sat(hi, c.D - c.L, shr_floor(lo, c.L));
  return shr_floor(hi + shr_floor(lo, c.D), c.L - c.D);
}

// floor(a 2^s) for a single term.
__device__ __forceinline__ int64_t scale1(int64_t a, int64_t s) {
  return s >= 0 ? shl_add_sat(a, s, 0) : shr_floor(a, -s);
}

// msb of the exact z* = hi 2^D + lo (D >= 0), |hi|, |lo| < 2^61.
__device__ __forceinline__ int msb_exact2(int64_t hi, int64_t lo, int64_t D) {
  if (D <= 64) {
    __int128 t = (__int128)((unsigned __int128)(__int128)hi << (int)D) + (__int128)lo;
    return msb128(t);
  }
  if (hi == 0) return msb64(lo);
  // msb(floor(v / 2^k)) = msb(v) - k whenever the quotient is not 0 or -1
  __int128 t = (__int128)((unsigned __int128)(__int128)hi << 64) + (__int128)shr_floor(lo, D - 64);
  return msb128(t) + (int)(D - 64);
}

// ------------------------------------------------------------ estimates --

// nu(gamma) = floor(log2 gamma) + 2 for the device-evaluated estimate, or
// sets *zero when gamma = 0.
// Metadata reads of an op go through an accessor: ma(k, f) is field f of
// operand k (kOpX, kOpY, kOpZ, or the estimate's blocks kOpGa, kOpGb).
enum { kOpX = 0, kOpY = 1, kOpZ = 2, kOpGa = 3, kOpGb = 4 };

// the operands' metadata in global memory, through the op's pointers
struct PtrMeta {
  const int64_t* p[5];
  __device__ __forceinline__ int64_t operator()(int k, int f) const { return p[k][f]; }
};

template <class MA>
__device__ __forceinline__ int64_t norm_mag(const MA& ma, int k) {
  const int64_t mx = ma(k, kMetaMax), mn = ma(k, kMetaMin);
  return mx > -mn ? mx : -mn;
}

template <class MA>
__device__ __forceinline__ int64_t gamma_nu(const GammaArgs& g, const MA& ma, bool* zero) {
  *zero = false;
  if (g.rule == kGammaNorm) {
    int64_t M = norm_mag(ma, kOpGa);
    if (M == 0) { *zero = true; return 0; }
    uint64_t prod = (uint64_t)M * (uint64_t)g.cm;
    return (int64_t)bitlen64(prod) + 1 + g.ce + ma(kOpGa, kMetaExp);
  }
  if (g.rule == kGammaSum) {
    int64_t Ma = norm_mag(ma, kOpGa), Mb = norm_mag(ma, kOpGb);
    int64_t ea = ma(kOpGa, kMetaExp), eb = ma(kOpGb, kMetaExp);
    if (Ma == 0 && Mb == 0) { *zero = true; return 0; }
    if (Ma == 0) return (int64_t)bitlen64((uint64_t)Mb) + 1 + eb;
    if (Mb == 0) return (int64_t)bitlen64((uint64_t)Ma) + 1 + ea;
    if (ea < eb) { int64_t t = Ma; Ma = Mb; Mb = t; t = ea; ea = eb; eb = t; }
    int64_t k = ea - eb;  // Ma carries the larger exponent
    if (k <= 31) return (int64_t)bitlen64(((uint64_t)Ma << k) + (uint64_t)Mb) + 1 + eb;
    // Mb <= 2^31 < 2^k: floor(log2(Ma 2^k + Mb)) = floor(log2 Ma) + k
    return (int64_t)bitlen64((uint64_t)Ma) + 1 + ea;
  }
  // explicit value c >= 0
  if (g.cm == 0) { *zero = true; return 0; }
  return (int64_t)msb64(g.cm) + g.ce;
}

// ------------------------------------------------ metadata reductions --

// Wave-wide reductions of 32-bit values with DPP (no LDS round trips): a
// scan within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row
// totals are carried forward (row_bcast 15 into rows 1 and 3, row_bcast 31
// into rows 2 and 3), so lane 63 ends with the reduction of all 64 lanes.
// Lanes whose DPP source is out of range read `id`, the identity.
template <typename F>
__device__ __forceinline__ int32_t wave_reduce32(int32_t v, int32_t id, F op) {
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int32_t wave_max32(int32_t v) {
  return wave_reduce32(v, INT32_MIN, [](int32_t a, int32_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ int32_t wave_min32(int32_t v) {
  return wave_reduce32(v, INT32_MAX, [](int32_t a, int32_t b) { return a < b ? a : b; });
}
__device__ __forceinline__ int32_t wave_sum32(int32_t v) {
  return wave_reduce32(v, 0, [](int32_t a, int32_t b) { return a + b; });
}

__device__ __forceinline__ int64_t wave_max(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(v, o, 64); v = t > v ? t : v; }
  return v;
}
__device__ __forceinline__ int64_t wave_min(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(v, o, 64); v = t < v ? t : v; }
  return v;
}
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------- grid reductions --
//
// A launch reduces per-block partials into accumulator sets in the output
// metadata and the last block to finish publishes the result and resets the
// sets. All cross-block traffic goes through device-scope atomic
// read-modify-writes (coherent across XCDs); a block's accumulator atomics
// return before it takes its ticket (s_waitcnt vmcnt(0)), so the block that
// draws the last ticket sees every contribution. No cache write-back or
// invalidation fence is needed, and the scratch is left ready for the next
// launch without a reset kernel.

__device__ __forceinline__ unsigned block_linear() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

__device__ __forceinline__ int64_t* acc_set(int64_t* meta) {
  return meta + kSetBase + kSetStride * (int)(block_linear() % kSets);
}

__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int64_t amax(int64_t* p, int64_t v) {
  return (int64_t)atomicMax((long long*)p, (long long)v);
}
__device__ __forceinline__ int64_t amin(int64_t* p, int64_t v) {
  return (int64_t)atomicMin((long long*)p, (long long)v);
}
__device__ __forceinline__ int64_t aadd(int64_t* p, int64_t v) {
  return (int64_t)atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ int64_t axch(int64_t* p, int64_t v) {
  return (int64_t)atomicExch((unsigned long long*)p, (unsigned long long)v);
}

// Returns true (in the calling thread) when this block finished last. The
// argument keeps the caller's accumulator atomics returning (their results
// are consumed), so the wait below covers them. Tickets are two-level: a
// block counts itself in its set; the last block of a set counts the set at
// the top level. One address never sees more than ~nblocks / kSets atomics.
// Grids of at most kOneLevel blocks count at the top level directly (one
// round trip fewer on the path of the last block).
constexpr unsigned kOneLevel = 2 * kSets;
__device__ __forceinline__ bool take_ticket(int64_t* meta, int64_t returned) {
  __shared__ volatile int64_t s_sink;
  s_sink = returned;
  wait_vmem();
  const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
  if (nblk <= kOneLevel) return (unsigned)aadd(&meta[kMetaTicket], 1) == nblk - 1;
  const unsigned b = block_linear();
  const unsigned k = b % kSets;
  const unsigned in_set = (nblk - k + kSets - 1) / kSets;          // blocks of set k
  const unsigned used = nblk < (unsigned)kSets ? nblk : (unsigned)kSets;
  int64_t* set = meta + kSetBase + kSetStride * (int)k;
  if ((unsigned)aadd(&set[kAccTicket], 1) != in_set - 1) return false;
  axch(&set[kAccTicket], 0);
  return (unsigned)aadd(&meta[kMetaTicket], 1) == used - 1;
}

__device__ __forceinline__ int64_t block_max(int64_t v, int64_t* red) {
  const int tid = threadIdx.x;
  v = wave_max(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  int64_t b = red[0];
  for (int i = 1; i < kBlock / 64; ++i) b = red[i] > b ? red[i] : b;
  return b;
}

// Diagnostic counts of a finished op (no-return atomics: nothing waits on
// them before the launch ends).
__device__ __forceinline__ void diag_count(int64_t* diag, int dbin, int dsat, int64_t nsat) {
  if (!diag) return;
  if (dbin >= 0) atomicAdd((unsigned long long*)&diag[dbin], 1ull);
  if (dsat) {
    atomicAdd((unsigned long long*)&diag[kDiagNnCalls], 1ull);
    if (nsat) {
      atomicAdd((unsigned long long*)&diag[kDiagNnSat], (unsigned long long)nsat);
      atomicAdd((unsigned long long*)&diag[kDiagNnSatCalls], 1ull);
    }
  }
}

// Reduce the per-thread (max, min, saturations) of a block's outputs; the
// last block publishes exponent / max / min / saturation count.
__device__ __forceinline__ void finish_outputs(int64_t tmax, int64_t tmin, int64_t tsat,
                                               int64_t* zm, int64_t e_out) {
  __shared__ int64_t s_red[3][kBlock / 64];
  const int tid = threadIdx.x;
  tmax = wave_max(tmax);
  tmin = wave_min(tmin);
  tsat = wave_sum(tsat);
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = tmax;
    s_red[1][tid >> 6] = tmin;
    s_red[2][tid >> 6] = tsat;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t bmax = s_red[0][0], bmin = s_red[1][0], bsat = s_red[2][0];
    for (int i = 1; i < kBlock / 64; ++i) {
      bmax = s_red[0][i] > bmax ? s_red[0][i] : bmax;
      bmin = s_red[1][i] < bmin ? s_red[1][i] : bmin;
      bsat += s_red[2][i];
    }
    if (gridDim.x * gridDim.y * gridDim.z == 1) {   // the block holds the whole result
      zm[kMetaMax] = bmax;
      zm[kMetaMin] = bmin;
      zm[kMetaSat] = bsat;
      zm[kMetaExp] = e_out;
      return;
    }
    int64_t* set = acc_set(zm);
    int64_t r = amax(&set[kAccMax], bmax) ^ amin(&set[kAccMin], bmin);
    if (bsat) r ^= aadd(&set[kAccSat], bsat);
    if (take_ticket(zm, r)) {
      int64_t mx = INT64_MIN, mn = INT64_MAX, st = 0;
      for (int k = 0; k < kSets; ++k) {
        int64_t* sk = zm + kSetBase + kSetStride * k;
        const int64_t a = axch(&sk[kAccMax], INT64_MIN);
        const int64_t b = axch(&sk[kAccMin], INT64_MAX);
        mx = a > mx ? a : mx;
        mn = b < mn ? b : mn;
        st += axch(&sk[kAccSat], 0);
      }
      axch(&zm[kMetaTicket], 0);
      zm[kMetaMax] = mx;
      zm[kMetaMin] = mn;
      zm[kMetaSat] = st;
      zm[kMetaExp] = e_out;
    }
  }
}

// First pass of qcomp: reduce mu* = max(1, max msb(z*_i)); the last block
// stores it in kMetaMu.
__device__ __forceinline__ void finish_mu(int64_t tmu, int64_t* zm) {
  __shared__ int64_t s_red[kBlock / 64];
  const int64_t b = block_max(tmu, s_red);
  if (threadIdx.x == 0 && gridDim.x * gridDim.y * gridDim.z == 1) {
    zm[kMetaMu] = b < 1 ? 1 : b;
    return;
  }
  if (threadIdx.x == 0) {
    int64_t* set = acc_set(zm);
    if (take_ticket(zm, amax(&set[kAccMu], b))) {
      int64_t mu = 1;
      for (int k = 0; k < kSets; ++k) {
        const int64_t a = axch(&zm[kSetBase + kSetStride * k + kAccMu], 0);
        mu = a > mu ? a : mu;
      }
      axch(&zm[kMetaTicket], 0);
      zm[kMetaMu] = mu;
    }
  }
}

// Reductions through per-block slots (a caller-provided array of 2 int64
// per block, e.g. one per solver hierarchy): thread 0 of every block
// exchanges its packed partial into its own slots (no two blocks touch the
// same address, so nothing queues behind other blocks' atomics), then
// takes the two-level ticket; in the block that finishes last, one wave
// reads all slots at once (independent atomics, one round trip) and
// publishes the result. Every slot [0, blocks) is written by each launch
// before its ticket, so no reset is needed.
__device__ __forceinline__ void finish_outputs_slots(int64_t tmax, int64_t tmin, int64_t tsat,
                                                     int64_t* zm, int64_t* slots, int64_t e_out) {
  __shared__ int32_t s_red[3][kBlock / 64];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int32_t a = wave_max32((int32_t)tmax), b = wave_min32((int32_t)tmin),
                c = wave_sum32((int32_t)tsat);
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = a;
    s_red[1][tid >> 6] = b;
    s_red[2][tid >> 6] = c;
  }
  __syncthreads();
  const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
  if (tid == 0) {
    int32_t bmax = s_red[0][0], bmin = s_red[1][0];
    int64_t bsat = s_red[2][0];
    for (int i = 1; i < kBlock / 64; ++i) {
      bmax = s_red[0][i] > bmax ? s_red[0][i] : bmax;
      bmin = s_red[1][i] < bmin ? s_red[1][i] : bmin;
      bsat += s_red[2][i];
    }
    if (nblk == 1) {
      zm[kMetaMax] = bmax;
      zm[kMetaMin] = bmin;
      zm[kMetaSat] = bsat;
      zm[kMetaExp] = e_out;
      s_last = 0;
    } else {
      const unsigned blk = block_linear();
      const uint64_t packed = ((uint64_t)(uint32_t)bmax << 32) | (uint32_t)bmin;
      const int64_t r = axch(&slots[2 * blk], (int64_t)packed) ^ axch(&slots[2 * blk + 1], bsat);
      s_last = take_ticket(zm, r);
    }
  }
  __syncthreads();
  if (!s_last || tid >= 64) return;
  int32_t mx = 0, mn = 0;
  int64_t st = 0;
  for (unsigned k = tid; k < nblk; k += 64) {
    const uint64_t p = (uint64_t)axch(&slots[2 * k], 0);
    const int32_t hmax = (int32_t)(uint32_t)(p >> 32), hmin = (int32_t)(uint32_t)p;
    mx = hmax > mx ? hmax : mx;
    mn = hmin < mn ? hmin : mn;
    st += axch(&slots[2 * k + 1], 0);
  }
  mx = wave_max32(mx);
  mn = wave_min32(mn);
  // the saturation count as two 32-bit DPP sums (its low 24 bits and the
  // rest; exact for counts below 2^55) instead of a chain of 64-bit shuffles
  const int32_t slo = wave_sum32((int32_t)(st & 0xFFFFFF)), shi = wave_sum32((int32_t)(st >> 24));
  st = ((int64_t)shi << 24) + slo;
  if (tid == 0) {
    axch(&zm[kMetaTicket], 0);
    zm[kMetaMax] = mx;
    zm[kMetaMin] = mn;
    zm[kMetaSat] = st;
    zm[kMetaExp] = e_out;
  }
}

// First qcomp pass through slots: mu* = max(1, max of the blocks' mu).
__device__ __forceinline__ void finish_mu_slots(int64_t tmu, int64_t* zm, int64_t* slots) {
  __shared__ int32_t s_red[kBlock / 64];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int32_t m = wave_max32((int32_t)tmu);
  if ((tid & 63) == 0) s_red[tid >> 6] = m;
  __syncthreads();
  const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
  if (tid == 0) {
    int32_t b = s_red[0];
    for (int i = 1; i < kBlock / 64; ++i) b = s_red[i] > b ? s_red[i] : b;
    if (nblk == 1) {
      zm[kMetaMu] = b < 1 ? 1 : b;
      s_last = 0;
    } else {
      s_last = take_ticket(zm, axch(&slots[2 * block_linear()], b));
    }
  }
  __syncthreads();
  if (!s_last || tid >= 64) return;
  int32_t mu = 1;
  for (unsigned k = tid; k < nblk; k += 64) {
    const int32_t v = (int32_t)axch(&slots[2 * k], 0);
    mu = v > mu ? v : mu;
  }
  mu = wave_max32(mu);
  if (tid == 0) {
    axch(&zm[kMetaTicket], 0);
    zm[kMetaMu] = mu;
  }
}

// --------------------------------------------------------- op planning --

// Everything a kernel derives once (uniformly) from the metadata of its
// operands: the exponents of the two exact terms a = alpha A x (exponent ea)
// and b = beta y (exponent eb), e_z* = min(ea, eb), the output exponent and
// the combine plan.
struct Resolved {
  int64_t ea, eb, ez, eo;
  Combine cmb;
  int64_t sa;    // single-term shift when there is no y
};

template <class MA>
__device__ __forceinline__ Resolved resolve(const OpArgs& p, const MA& ma) {
  Resolved r;
  r.ea = p.alpha_e + p.e_A + ma(kOpX, kMetaExp);
  r.eb = p.has_y ? p.beta_e + ma(kOpY, kMetaExp) : r.ea;
  r.ez = r.ea < r.eb ? r.ea : r.eb;
  if (p.mode == kModeSat) {
    bool zero;
    int64_t nu = gamma_nu(p.g, ma, &zero);
    r.eo = zero ? r.ez + 1 - p.w_out : nu - p.w_out;
  } else if (p.mode == kModeQ2) {
    r.eo = r.ez + ma(kOpZ, kMetaMu) - p.w_out;
  } else if (p.mode == kModeNormMeta) {
    // mu* of a stored block from its max / min (msb is monotone in |v|)
    int64_t a = msb64(ma(kOpX, kMetaMax)), b = msb64(ma(kOpX, kMetaMin));
    r.eo = r.ez + (a > b ? a : b) - p.w_out;
  } else if (p.mode == kModeAssign) {
    r.eo = p.assign_exp;
  } else {
    r.eo = 0;
  }
  r.sa = p.mode == kModeAssign ? 0 : r.ea - r.eo;
  r.cmb = make_combine(r.ea - r.eo, r.eb - r.eo);
  return r;
}

__device__ __forceinline__ PtrMeta ptr_meta(const OpArgs& p) {
  return PtrMeta{{p.x_meta, p.y_meta, p.z_meta, p.g.a, p.g.b}};
}

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi, int64_t& sat) {
  if (v < lo) { ++sat; return lo; }
  if (v > hi) { ++sat; return hi; }
  return v;
}

}  // namespace bfpk
