// Internal helpers of the C-ABI layer shared with the multigrid driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bfpmg.h"
#include "common.hpp"
#include "kernels.hpp"

#include <vector>

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

// The launch description of a star op in saturate mode (the checks and
// preparation of stencil_apply_impl), without launching it; outside a
// recording only.
int star_prepare_sat(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                     const bfp_scalar* beta, const bfp_vec* y, int w_out,
                     const bfp_gamma* gamma, bfp_vec* z, StarLaunch* out);

// forced_mode = kModeNormMeta selects the one-pass normalization of a stored
// block; -1 follows `mode`.
int point_impl(const bfp_scalar* alpha, const bfp_vec* x, const bfp_scalar* beta,
               const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma, bfp_vec* z,
               hipStream_t s, int forced_mode);

// Recording of coarse-level programs: while a sink is installed on the
// calling thread, stencil_apply_impl, point_impl and bfp_vec_init append
// ExecOps to it instead of launching kernels.
void record_into(std::vector<ExecOp>* sink);
bool recording();
// Diagnostic counters (kDiagBins) that the next operations issued on this
// host thread count into; null turns the counting off.
void set_diag_row(int64_t* row);
// Per-block reduction slots (2 * kMaxSlotBlocks int64) the next operations
// issued on this host thread use; null: the output's accumulator sets.
void set_slots(int64_t* slots);
// Whether hierarchies created now keep diagnostics (tuning key "diagnostics").
bool diagnostics_on();
// grids of at most this many points run inside recorded programs (0: never)
int exec_max_points();
// plain streaming copy of `bytes` (a multiple of 16, 16-byte aligned)
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, bool nontemporal,
                              int max_blocks, int per_thread, hipStream_t s);
// the V-cycle's relaxation and residual in one launch where they fit it
// (tuning key "fuse_relax_res", default off) on grids up to
// "relax_res_max_n" points a side, and its rows per wave ("relax_res_rows";
// 0: automatic)
bool fuse_relax_res();
// finite-element ops with at most this many outputs take both qcomp passes
// in one single-workgroup launch (tuning key "fe_one_launch"; 0: never)
int fe_one_launch();
// a finite-element FMG runs as its recorded single-workgroup program when
// the hierarchy has one (tuning key "fe_program", default on)
bool fe_program();
int relax_res_rows();
int relax_res_max_n();
// rows per wave of the 2D tiled stencil kernel (tuning key "tiles2d_rows"; 0: automatic)
int tiles_rows();
// Give every op of a recorded program the slots of its metadata blocks in
// the program's table of distinct blocks (filled into `metas`).
int exec_assign_slots(std::vector<ExecOp>& ops, std::vector<int64_t*>& metas);

// FP64 <-> BFP with the FP64 pointer given directly, or (pointer null) read
// on the device from table[index]
int from_f64_impl(const double* src_dev, const double* const* table_dev, int index,
                  int64_t log2_scale, bfp_vec* dst, hipStream_t s);
int to_f64_impl(const bfp_vec* src, double* dst_dev, double* const* table_dev, int index,
                hipStream_t s);
// mg_set_rhs with the level's FP64 right-hand side read from table[index]
int set_rhs_table(mg_hierarchy* h, int level, const double* const* table_dev, int index,
                  hipStream_t s);

// mg_hierarchy_bytes / mg_hierarchy_create with an explicit executor
// threshold (largest grid, in points, run inside recorded programs)
int hierarchy_bytes_ex(const mg_params* prm, int64_t exec_points, size_t* bytes);
int hierarchy_create_ex(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                        int64_t exec_points, mg_hierarchy** out);

// Chebyshev coefficients c1, c2, c1_gamma of p for eta = eta_percent / 100
// (rho = 2, rescaled to the stored operator, 16-bit)
int set_smoother(mg_params* p, int eta_percent);

// Per-level launch shapes (kind 0: star stencils, rows / planes per wave;
// kind 1: grid transfers, coarse rows / planes per wave, keyed by the fine
// level); 0 restores the default.
void set_level_rows(int kind, int ndim, int level, int rows);
int level_rows(int kind, int ndim, int level);

// mg_fmg_f64 on one stream (no side stream), same results
int fmg_f64_one_stream(mg_hierarchy* h, const double* const* rhs_dev, hipStream_t s);

// validation of multigrid parameters (BFP_OK or the error of mg_params checks)
int params_ok(const mg_params* p);

}  // namespace bfpk
