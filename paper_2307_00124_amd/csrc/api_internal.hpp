// Internal helpers of the C-ABI layer shared with the multigrid driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bfpmg.h"
#include "common.hpp"

namespace bfpk {

int fail(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
int64_t pitch_for(int64_t n, int bits);
int64_t rows_for(int ndim, int64_t n);
int check_vec(const bfp_vec* v, const char* name);

// rows: rows (2D) / planes (3D) marched per wave by the star kernels (0 = default)
int stencil_apply_impl(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                       const bfp_scalar* beta, const bfp_vec* y, int w_out, int mode,
                       const bfp_gamma* gamma, bfp_vec* z, hipStream_t s, int rows);

// forced_mode = kModeNormMeta selects the one-pass normalization of a stored
// block; -1 follows `mode`.
int point_impl(const bfp_scalar* alpha, const bfp_vec* x, const bfp_scalar* beta,
               const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma, bfp_vec* z,
               hipStream_t s, int forced_mode);

}  // namespace bfpk
