// Host-side launch descriptions of the BFP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace bfpk {

// Vector loads / stores of four consecutive mantissas.
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T v[4];
};

// z = Q(alpha * A x + beta * y) for a star stencil (center + 2*ndim faces)
// on one grid. taps: center, -x, +x, -y, +y, -z, +z.
struct StarLaunch {
  OpArgs op;
  const void* x;
  const void* y;
  void* z;
  int ndim;
  int64_t n;
  int64_t px, py, pz;
  int32_t taps[7];
  int xbits, ybits, zbits;
  int wide;   // 1: accumulate the stencil sum in int64
  int rows;   // rows (2D) or planes (3D) marched by one wave
  int wx;     // 2D: column segments per block (1, 2 or 4; the block's 4 waves
              // cover wx segments times 4 / wx row bands)
  int y_is_x; // y is the block x itself (the relaxation c2 A r + c1 r): its
              // entries are the centre values already loaded, not a stream
};
hipError_t launch_star(const StarLaunch& L, hipStream_t s);

// Restriction (fine n_f -> coarse n_c = (n_f - 1) / 2) with full 3^d taps,
// or prolongation (coarse -> fine) with full 3^d taps on the upsampled grid.
struct TransferLaunch {
  OpArgs op;
  int kind;        // 1 = R, 2 = P
  const void* x;   // input grid (fine for R, coarse for P)
  const void* y;   // on the output grid (may be null)
  void* z;         // output grid
  int ndim;
  int64_t n_in, n_out;
  int64_t px, py, pz;
  int32_t taps[27];
  int xbits, ybits, zbits;
  int rows;        // coarse rows (2D) or coarse planes (3D) one wave marches
};
hipError_t launch_transfer(const TransferLaunch& L, hipStream_t s);

// Pointwise z = Q(alpha x + beta y) on one grid (y optional).
struct PointLaunch {
  OpArgs op;
  const void* x;
  const void* y;
  void* z;
  int ndim;
  int64_t n;
  int64_t px, py, pz;
  int xbits, ybits, zbits;
};
hipError_t launch_point(const PointLaunch& L, hipStream_t s);

// Diagnostics of a launched operation with op.diag set: the qcomp window
// gap (launched between the two passes) or the nnqcomp saturations
// (launched after the operation, reading its output metadata zm).
hipError_t launch_diag_q(const OpArgs& op, hipStream_t s);
hipError_t launch_diag_sat(int64_t* diag, const int64_t* zm, hipStream_t s);

// FP64 <-> BFP conversion, initialisation and the exact dot product.
struct ConvertLaunch {
  const double* src;   // dense (n+2)^ndim
  double* dst;
  // when src (from_f64) or dst (to_f64) is null, the FP64 pointer is read
  // on the device from table[index] (lets a captured graph serve requests
  // whose buffers change)
  const double* const* src_table;
  double* const* dst_table;
  int table_index;
  void* mant;
  int64_t* meta;
  int ndim;
  int64_t n, pitch;
  int bits, w;
  int64_t log2_scale;
};
hipError_t launch_from_f64(const ConvertLaunch& L, hipStream_t s);
hipError_t launch_to_f64(const ConvertLaunch& L, hipStream_t s);
hipError_t launch_init(void* mant, size_t bytes, int64_t* meta, int64_t exp, hipStream_t s);
hipError_t launch_meta_reset(int64_t* meta, hipStream_t s);
// turn a zero block (bfp_vec_init) of width w into the unit vector e_pos:
// mantissa 2^(w-2) at element pos, exponent 2 - w
hipError_t launch_unit(void* mant, int bits, int64_t pos, int64_t* meta, int w, hipStream_t s);
// initialise count metadata blocks (exponent exps[i], identities elsewhere)
hipError_t launch_meta_init_list(int64_t* const* metas_dev, const int64_t* exps_dev, int count,
                                 hipStream_t s);

struct DotLaunch {
  const void* x;
  const void* y;
  const int64_t* x_meta;
  const int64_t* y_meta;
  int64_t* out;
  int ndim;
  int64_t n, px, py;
  int xbits, ybits;
};
hipError_t launch_dot(const DotLaunch& L, hipStream_t s);

// One recorded operation of a coarse-level program (see k_exec.hip): the
// launch description the library would otherwise launch, and its mode.
constexpr int kExStar = 1, kExTransfer = 2, kExPoint = 3, kExZero = 4, kExConv = 5;
constexpr int kExModeQ = 9;   // both qcomp passes, executed back to back

// bfp_vec_init inside a program: zero mantissas, exponent 1 - w
struct ZeroOp {
  void* mant;
  int64_t* meta;
  int64_t bytes;   // multiple of 16
  int64_t exp;
};

// bfp_vec_from_f64 inside a program: the FP64 source is `src`, or, when
// src is null, entry `level` - 1 of the running problem's right-hand-side
// table (batched solves)
struct ConvOp {
  const double* src;
  void* mant;
  int64_t* meta;
  int ndim;
  int64_t n, pitch;
  int bits, w;
  int64_t log2_scale;
  int level;
};

struct ExecOp {
  int kind;
  int mode;   // kModeSat, kModeNormMeta, kModeAssign or kExModeQ
  // metadata slots (x, y, z, gamma a, gamma b; -1 = none) in the program's
  // table of distinct metadata blocks, which the executor mirrors in LDS
  int16_t slot[5];
  union {
    StarLaunch star;
    TransferLaunch tr;
    PointLaunch pt;
    ZeroOp zero;
    ConvOp conv;
  } u;
};

// Run ops[0..count) in order inside one workgroup of kExecThreads threads;
// every op works on grids of one dimension ndim with n_out < kExecMaxN.
// metas[0..nmeta) are the metadata blocks the ops name by slot: the
// executor works on an LDS copy of their first kExMetaF fields and writes
// it back at the end.
constexpr int kExecThreads = 512;
constexpr int kExecMaxN = 1024;
constexpr int kExecMaxMeta = 64;
constexpr int kExMetaF = 8;
// rhs: the FP64 right-hand sides of levels 1..kMaxLevels (device pointers,
// passed by value in the launch) that the program's conversions read; may
// be null when the program has none.
struct ExecRhs {
  const double* p[16];
};
// diag: some ops of the program count diagnostics (their OpArgs::diag)
hipError_t launch_exec(const ExecOp* ops_dev, int count, int64_t* const* metas_dev, int nmeta,
                       int ndim, const ExecRhs* rhs, bool diag, hipStream_t s);

// Batched programs: one workgroup of kBatchThreads threads per problem runs
// that problem's program. Programs are relocatable: every data and metadata
// pointer in their ops and metadata tables is an offset from the problem's
// arena base. rhs_table[p * kMaxLevels + j - 1] is problem p's FP64
// right-hand side on level j.
constexpr int kBatchThreads = 256;
constexpr int kMaxLevels = 16;
static_assert(sizeof(ExecRhs) == kMaxLevels * sizeof(const double*), "one pointer per level");
struct BatchEntry {
  uintptr_t base;        // the problem's arena base
  int prob;              // row of the right-hand-side table
  int op_begin, op_count;
  int meta_begin, nmeta; // the program's metadata table (offsets)
};
hipError_t launch_exec_batch(const BatchEntry* entries_dev, int nentries, const ExecOp* ops_dev,
                             int64_t* const* metas_dev, const double* const* rhs_table_dev,
                             int ndim, hipStream_t s);

}  // namespace bfpk
