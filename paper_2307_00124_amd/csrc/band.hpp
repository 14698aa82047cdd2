// Banded matrix times a 1D block (the finite-element operators).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace bfpk {

// Output point i (padded index 1 + i) takes sum_k taps[i * band + k]
// x[1 + col0[i] + k]; taps == nullptr is the identity (pointwise rows).
// All blocks in int32 storage.
struct BandLaunch {
  OpArgs op;
  const int32_t* x;
  const int32_t* y;
  int32_t* z;
  int64_t nout;
  const int32_t* col0;
  const int32_t* taps;
  int band;
};
hipError_t launch_band(const BandLaunch& L, hipStream_t s);
// Both passes of qcomp (mode ignored) in one single-workgroup launch; only
// for nout <= kBandOneMax (hipErrorInvalidValue otherwise).
constexpr int64_t kBandOneMax = 16 * kBlock;
hipError_t launch_band_qcomp1(const BandLaunch& L, hipStream_t s);

}  // namespace bfpk
