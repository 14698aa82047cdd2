// The quantizing epilogue every BFP kernel applies to its exact per-point
// result, and vector load/store helpers.
//
// For an exact stencil row sum g (or a stored mantissa, for pointwise ops)
// and an optional y entry, the exact result is z* = a 2^ea + b 2^eb with
// a = alpha_m * g and b = beta_m * y (the exact gemv / axpby rows of the
// paper's Appendix B, with the operand of larger exponent shifted left).
//   - first qcomp pass (kQ1): accumulate mu* = max msb(z*) (z* held exactly
//     in 128 bits);
//   - every other mode: write floor(z* 2^(e_z* - e_out)) clamped to X_w_out,
//     with e_out fixed by the mode (estimate, mu*, or the input's metadata),
//     and accumulate max / min / saturation count of the outputs.
#pragma once

#include "device.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace bfpk {

constexpr int kQ1 = 1;   // template flag: first qcomp pass
constexpr int kOut = 0;  // template flag: output-writing pass (mode chosen at run time)

// Branch-free loads: an out-of-range request reads element 0 of the block
// (always valid) and yields zeros, so a batch of loads stays one straight
// run of instructions with no wait between them.
template <typename T>
__device__ __forceinline__ void ld4(const T* base, int64_t off, int32_t (&v)[4], bool ok) {
  const Q4<T> q = *reinterpret_cast<const Q4<T>*>(base + (ok ? off : 0));
  v[0] = ok ? (int32_t)q.v[0] : 0;
  v[1] = ok ? (int32_t)q.v[1] : 0;
  v[2] = ok ? (int32_t)q.v[2] : 0;
  v[3] = ok ? (int32_t)q.v[3] : 0;
}

template <typename T>
__device__ __forceinline__ int32_t ld1(const T* base, int64_t off, bool ok) {
  const T q = base[ok ? off : 0];
  return ok ? (int32_t)q : 0;
}

template <typename T>
__device__ __forceinline__ void st4(T* base, int64_t off, const int64_t (&v)[4]) {
  Q4<T> q;
  q.v[0] = (T)v[0]; q.v[1] = (T)v[1]; q.v[2] = (T)v[2]; q.v[3] = (T)v[3];
  *reinterpret_cast<Q4<T>*>(base + off) = q;
}

// Streaming variants for data touched once (the y operand, the output):
// non-temporal hints keep it from displacing re-used lines (stencil halos)
// in the caches. Measured on MI355X: a few percent faster for the 3D star
// kernel, slower for the 2D one (which therefore keeps plain accesses).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef int32_t v2i32 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void ld4_nt(const T* base, int64_t off, int32_t (&v)[4], bool ok) {
  const T* p = base + (ok ? off : 0);
  int32_t w[4];
  if (sizeof(T) == 4) {
    const v4i32 q = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(p));
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if (sizeof(T) == 2) {
    const v2i32 q = __builtin_nontemporal_load(reinterpret_cast<const v2i32*>(p));
    w[0] = (int16_t)(q.x & 0xffff); w[1] = (int16_t)((uint32_t)q.x >> 16);
    w[2] = (int16_t)(q.y & 0xffff); w[3] = (int16_t)((uint32_t)q.y >> 16);
  } else {
    const int q = __builtin_nontemporal_load(reinterpret_cast<const int*>(p));
    w[0] = (int8_t)(q & 0xff); w[1] = (int8_t)((q >> 8) & 0xff);
    w[2] = (int8_t)((q >> 16) & 0xff); w[3] = (int8_t)((uint32_t)q >> 24);
  }
  v[0] = ok ? w[0] : 0;
  v[1] = ok ? w[1] : 0;
  v[2] = ok ? w[2] : 0;
  v[3] = ok ? w[3] : 0;
}

template <typename T>
__device__ __forceinline__ void st4_nt(T* base, int64_t off, const int64_t (&v)[4]) {
  T* p = base + off;
  if (sizeof(T) == 4) {
    const v4i32 q = {(int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<v4i32*>(p));
  } else if (sizeof(T) == 2) {
    const v2i32 q = {(int32_t)((uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16)),
                     (int32_t)((uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16))};
    __builtin_nontemporal_store(q, reinterpret_cast<v2i32*>(p));
  } else {
    const int q = (int)((uint32_t)(uint8_t)v[0] | ((uint32_t)(uint8_t)v[1] << 8) |
                        ((uint32_t)(uint8_t)v[2] << 16) | ((uint32_t)(uint8_t)v[3] << 24));
    __builtin_nontemporal_store(q, reinterpret_cast<int*>(p));
  }
}

// Epilogue variants chosen once per launch, outside the loops:
//   kVarFastA1 — fast path and alpha = 1 (a = g, no multiply),
//   kVarFast   — fast path, general alpha,
//   kVarGen    — exact generic combine.
constexpr int kVarGen = 0, kVarFast = 1, kVarFastA1 = 2;

template <typename E, typename F>
__device__ __forceinline__ void with_fast(const E& e, F&& body) {
  if (e.fast && e.alpha_m == 1) body(std::integral_constant<int, kVarFastA1>());
  else if (e.fast) body(std::integral_constant<int, kVarFast>());
  else body(std::integral_constant<int, kVarGen>());
}

// DG = true: the executor's programs that count diagnostics (the op's
// counts are prepared at set-up). Launched operations are counted by small
// kernels of their own (k_diag_q, k_diag_sat), so these carry no
// diagnostic state at all.
template <int PASS, bool HASY, bool DG = false>
struct Epi {
  Resolved R;
  int64_t alpha_m, beta_m, lo, hi;
  int64_t D;       // first pass: exponent gap of the two terms
  int swap;        // first pass: the y term carries the larger exponent
  // Fast path, exact whenever no intermediate can overflow: with la, lb the
  // shifts that bring the terms to the output exponent (la = ea - eo) and
  // h / l the term with the larger / smaller shift,
  //   both <= 0:  floor(h 2^sh + l 2^sl) = (h + (l >> (sh - sl))) >> -sh
  //   sh >= 0:    floor(h 2^sh + l 2^sl) = (h << sh) + floor(l 2^sl)
  // so one expression ((h << fa) + ((l << fb) >> fc)) >> fs covers both;
  // the second case is taken only when |h| 2^sh and |l| 2^max(sl,0) stay
  // below 2^62 (bit bounds from the host), else the generic combine runs.
  int fast;
  int fswap, fa, fb, fc, fs;
  int32_t tsat;
  int32_t tmax, tmin;
  int64_t tmu;
  int64_t* zm;
  int64_t* slots;  // per-block partials of the reduction (or null)
  int64_t* diag;   // the call site's diagnostic counters (or null)
  int dbin;        // qcomp window-gap bin to count, or -1
  int dsat;        // 1: count an nnqcomp call and its saturations

  __device__ __forceinline__ void init(const OpArgs& op) { init(op, ptr_meta(op)); }

  template <class MA>
  __device__ __forceinline__ void init(const OpArgs& op, const MA& ma) {
    R = resolve(op, ma);
    alpha_m = op.alpha_m;
    beta_m = op.beta_m;
    lo = op.lo;
    hi = op.hi;
    zm = op.z_meta;
    slots = op.slots;
    swap = R.ea < R.eb;
    D = swap ? R.eb - R.ea : R.ea - R.eb;
    const int64_t la = R.sa, lb = R.eb - R.eo;
    auto c63 = [](int64_t v) { return (int)(v > 63 ? 63 : v); };
    if (HASY) {
      fswap = la < lb;
      const int64_t sh = fswap ? lb : la, sl = fswap ? la : lb;
      const int hb = fswap ? op.bbits : op.abits, lb_bits = fswap ? op.abits : op.bbits;
      if (sh <= 0) {
        fast = 1;
        fa = 0;
        fb = 0;
        fc = c63(sh - sl);
        fs = c63(-sh);
      } else {
        fa = (int)(sh > 62 ? 62 : sh);
        fb = sl > 0 ? (int)sl : 0;
        fc = sl < 0 ? c63(-sl) : 0;
        fs = 0;
        fast = hb + sh <= 62 && lb_bits + fb <= 62;
      }
    } else {
      fswap = 0;
      fb = 0;
      fc = 0;
      if (la <= 0) {
        fast = 1;
        fa = 0;
        fs = c63(-la);
      } else {
        fa = (int)(la > 62 ? 62 : la);
        fs = 0;
        fast = op.abits + la <= 62;
      }
    }
    // first qcomp pass: z* = h 2^D + l (h the term of larger exponent) fits
    // int64 when |h| 2^D < 2^62 (bit bound of h from the host, |l| < 2^61),
    // so its msb needs no 128-bit arithmetic
    if (PASS == kQ1 && HASY) fast = (swap ? op.bbits : op.abits) + D <= 62;
    if (PASS == kQ1 && !HASY) fast = 1;
    tmax = 0;
    tmin = 0;
    tsat = 0;
    tmu = 1;
    // diagnostics: the window gap of a qcomp call with an estimate (the
    // second pass knows mu* = eo - ez + w_out), or an nnqcomp call
    diag = DG ? op.diag : nullptr;
    dbin = -1;
    dsat = 0;
    if (DG && diag) {   // off the common path: only hierarchies that keep diagnostics
      if (op.mode == kModeQ2) {
        bool zero;
        const int64_t nu = gamma_nu(op.g, ma, &zero);
        // mu* = eo - ez + w_out in the second qcomp pass
        if (!zero) dbin = diag_gap_bin(nu - R.ez - (R.eo - R.ez + op.w_out));
      }
      dsat = op.mode == kModeSat;
    }
  }

  __device__ __forceinline__ int64_t mul_a(int64_t g) const { return alpha_m * g; }
  // |beta| < 2^31 (checked on the host): one 32 x 32 -> 64-bit multiply
  __device__ __forceinline__ int64_t mul_b(int32_t y) const {
    return (int64_t)(int32_t)beta_m * (int64_t)y;
  }

  // floor of the exact result at the output exponent (+-2^62 when beyond);
  // VAR must match the launch (the kernels choose it once via with_fast)
  template <int VAR>
  __device__ __forceinline__ int64_t value(int64_t g, int32_t yv) const {
    const int64_t a = VAR == kVarFastA1 ? g : mul_a(g);
    if (!HASY) return VAR != kVarGen ? ((a << fa) >> fs) : scale1(a, R.sa);
    const int64_t b = mul_b(yv);
    if (VAR != kVarGen) {
      const int64_t h = fswap ? b : a, l = fswap ? a : b;
      return ((h << fa) + ((l << fb) >> fc)) >> fs;
    }
    return combine(R.cmb, a, b);
  }

  // Process one output point (inside = interior point of the output grid);
  // returns its mantissa, 0 outside or in the first qcomp pass.
  template <int VAR>
  __device__ __forceinline__ int64_t put(int64_t g, int32_t yv, bool inside) {
    if (PASS == kQ1) {
      const int64_t a = VAR == kVarFastA1 ? g : mul_a(g);
      int m;
      if (HASY) {
        const int64_t b = mul_b(yv);
        const int64_t h = swap ? b : a, l = swap ? a : b;
        if (VAR != kVarGen) m = msb64((int64_t)((uint64_t)h << (int)D) + l);
        else m = msb_exact2(h, l, D);
      } else {
        m = msb64(a);
      }
      m = inside ? m : 1;
      tmu = m > tmu ? m : tmu;
      return 0;
    }
    const int64_t v = value<VAR>(g, yv);
    const int64_t c = v < lo ? lo : (v > hi ? hi : v);
    tsat += (inside && c != v) ? 1 : 0;
    const int32_t r = inside ? (int32_t)c : 0;
    tmax = r > tmax ? r : tmax;
    tmin = r < tmin ? r : tmin;
    return r;
  }

  __device__ __forceinline__ void finish() {
    if (slots) {
      if (PASS == kQ1) finish_mu_slots(tmu, zm, slots);
      else finish_outputs_slots(tmax, tmin, tsat, zm, slots, R.eo);
      return;
    }
    if (PASS == kQ1) finish_mu(tmu, zm);
    else finish_outputs(tmax, tmin, tsat, zm, R.eo);
  }

};

// Storage-type dispatch helpers (host side).
template <typename F>
inline hipError_t with_type(int bits, F&& f) {
  switch (bits) {
    case 8: return f((int8_t)0);
    case 16: return f((int16_t)0);
    case 32: return f((int32_t)0);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bfpk
