// Constants and kernel argument blocks shared by the host launchers and the
// HIP kernels of the BFP library.
#pragma once

#include <stdint.h>

namespace bfpk {

constexpr int kBlock = 256;       // threads per workgroup for every kernel
constexpr int kMaxBlocks = 2048;  // grid-stride kernels launch at most this many

// metadata slots (see include/bfpmg.h); 16.. are reduction scratch: a
// top-level ticket and kSets accumulator sets (max, min, saturations, mu*,
// set ticket), each set in its own 128-byte line; a block uses set
// (linear block index mod kSets), which spreads a launch's atomics over
// kSets addresses.
constexpr int kMetaExp = 0, kMetaMax = 1, kMetaMin = 2, kMetaSat = 3, kMetaMu = 4,
              kMetaFlags = 5;
constexpr int kMetaTicket = 16;
constexpr int kSets = 16, kSetBase = 32, kSetStride = 16;
constexpr int kAccMax = 0, kAccMin = 1, kAccSat = 2, kAccMu = 3, kAccTicket = 4;  // in a set
constexpr int kMetaSlots = kSetBase + kSets * kSetStride;           // 288

constexpr int kGammaNorm = 1, kGammaSum = 2, kGammaExplicit = 3;

// Diagnostics of one (level, call site) of a solve: 64 counters.
//   bins 0..60: qcomp calls with an estimate, by the window gap
//     d = mu_tmp - mu* (mu_tmp = nu(gamma) - e_z*, the top of the window the
//     estimate gives; Algorithm 1 recomputes when d < 0 — overflow — or when
//     d > w_tmp - w_out — underflow): bin 0 for d < 0, bin 1 + min(d, 59);
//   bin 61: nnqcomp calls; bin 62: entries they saturated; bin 63: nnqcomp
//   calls that saturated at least one entry.
constexpr int kDiagBins = 64, kDiagGapBins = 61, kDiagNnCalls = 61, kDiagNnSat = 62,
              kDiagNnSatCalls = 63;
__host__ __device__ inline int diag_gap_bin(int64_t d) {
  return d < 0 ? 0 : 1 + (int)(d < kDiagGapBins - 2 ? d : kDiagGapBins - 2);
}

// kModeSat: nnqcomp; kModeQ1 / kModeQ2: the two passes of qcomp;
// kModeNormMeta: qcomp of a stored block whose mu* is known from its metadata;
// kModeAssign: keep the mantissas, set the exponent, recompute the metadata
constexpr int kModeSat = 0, kModeQ1 = 1, kModeQ2 = 2, kModeNormMeta = 3, kModeAssign = 4;

struct GammaArgs {
  int rule;
  const int64_t* a;
  const int64_t* b;
  int64_t cm, ce;
};

// One quantized BFP operation z = Q(alpha * S x + beta * y).
struct OpArgs {
  int mode;
  int has_y;
  int w_out;
  int64_t e_A;              // exponent of the stencil (0 for pointwise ops)
  int64_t alpha_m, alpha_e;
  int64_t beta_m, beta_e;
  const int64_t* x_meta;
  const int64_t* y_meta;
  int64_t* z_meta;
  GammaArgs g;
  int64_t lo, hi;           // X_w_out
  int64_t assign_exp;       // kModeAssign only
  int abits, bbits;         // |alpha S x| < 2^abits and |beta y| < 2^bbits
  int64_t* diag;            // kDiagBins diagnostic counters of the op's call site, or null
  int64_t* slots;           // 2 * kMaxSlotBlocks int64 of per-block partials for the
                            // output reduction, or null (z's accumulator sets)
};

// Launches with at most this many blocks may reduce through per-block slots.
constexpr int kMaxSlotBlocks = 8192;

// A padded, row-pitched grid: rows = (n+2)^(ndim-1) rows of `pitch` elements.
struct Grid {
  int64_t n;       // interior points per dimension
  int64_t pitch;   // elements per row
};

}  // namespace bfpk
