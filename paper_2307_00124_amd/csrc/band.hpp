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

// One step of a recorded finite-element program: a band op (both qcomp
// passes, nout <= kBandOneMax, u = ceil(nout / kBlock)), or, with init_meta
// set, the initialisation of a block (init_words int32 mantissas zeroed,
// metadata set to exponent init_exp and the reduction identities).
struct BandStep {
  BandLaunch L;
  int u;
  int32_t* init_mant;
  int64_t init_words;
  int64_t* init_meta;
  int64_t init_exp;
};
// Runs the nsteps steps (device array) in order in one single-workgroup
// launch.
hipError_t launch_band_prog(const BandStep* steps, int nsteps, hipStream_t s);

}  // namespace bfpk
