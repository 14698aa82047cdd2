/*
 * bfpmg.h — block-floating-point (BFP) vector operations and multigrid on
 * AMD MI355X (gfx950).
 *
 * Method: N. Kohl, S. F. McCormick, R. Tamstorf, "Multigrid methods using
 * Block Floating Point Arithmetic". A BFP block is the tuple (e, m, w, d) of
 * Section 2: one shared integer exponent e for a whole vector or matrix and
 * w-bit two's-complement integer mantissas m, representing 2^e * m. Right
 * shifts round toward minus infinity (floor).
 *
 * Conventions for every function below
 *   - Return value: BFP_OK (0) or a negative bfp_status; BFP_PENDING (1) only
 *     from mg_server_poll. bfp_last_error() describes the last failure of the
 *     calling thread. No exception crosses this interface.
 *   - Pointers named *_dev, bfp_vec.mant and bfp_vec.meta are device pointers
 *     owned by the caller; the library never frees caller memory. Host
 *     structs are read during the call only and may be reused afterwards.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every operation is asynchronous on that stream; exponents, norms and
 *     estimates stay in device memory, so no call below synchronizes with
 *     the host except where stated.
 *   - Shape, width and argument errors are detected on the host before any
 *     launch; on error nothing is enqueued and nothing is written.
 *   - Calls that write the same block must not overlap in time (different
 *     streams without ordering); blocks that are only read may be shared.
 */
#ifndef BFPMG_H
#define BFPMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BFP_OK = 0,
  BFP_EINVAL = -1,     /* bad argument (null pointer, bad enum, aliasing)      */
  BFP_EWIDTH = -2,     /* width outside 1..storage bits, or an exact product   */
                       /* that could exceed the 62-bit integer budget          */
  BFP_ESHAPE = -3,     /* grids of incompatible size / layout                  */
  BFP_ENONFINITE = -4, /* NaN or Inf in FP64 input (reported by bfp_vec_check) */
  BFP_ENOMEM = -5,     /* arena too small                                      */
  BFP_EHIP = -6,       /* a HIP runtime call failed                            */
  BFP_EBUSY = -7,      /* server admission queue full                          */
  BFP_ENOTFOUND = -8,  /* unknown ticket                                       */
  BFP_PENDING = 1      /* request not finished yet                             */
} bfp_status;

/* How an exact result z* is quantized to w_out bits (1 <= w_out <= the
 * width w of the output block, which then holds w_out-bit mantissas).
 *  BFP_NORMALIZE — qcomp (Algorithm 1): normalized result, exact up to w_out
 *     bits: e_out = e_z* + mu* - w_out with mu* = max(1, max_i msb(z*_i)),
 *     m_i = floor(z*_i / 2^(mu* - w_out)). Independent of any estimate.
 *     Implemented as two passes over the inputs (the "compute twice"
 *     strategy of Section 4): the first finds mu*, the second writes.
 *  BFP_SATURATE — nnqcomp (Algorithm 3): e_out = floor(log2 gamma) + 2 - w_out
 *     from the estimate gamma alone, m_i = clamp(floor(z*_i 2^(e_z*-e_out)),
 *     X_w_out). One pass. A zero gamma gives e_out = e_z* + 1 - w_out. */
typedef enum { BFP_NORMALIZE = 0, BFP_SATURATE = 1 } bfp_mode;

/* Device metadata of a block: BFP_META_SLOTS int64 values (2304 bytes).
 *   [BFP_META_EXP] shared exponent e
 *   [BFP_META_MAX] largest mantissa, [BFP_META_MIN] smallest mantissa
 *                  (both taken over the whole padded array, ring included,
 *                  so MAX >= 0 >= MIN and ||x||_inf = max(MAX, -MIN) * 2^e)
 *   [BFP_META_SAT] entries saturated by the operation that wrote the block
 *   [BFP_META_MU]  mu* of the last BFP_NORMALIZE operation writing the block
 *   [BFP_META_FLAGS] bit 0: non-finite FP64 input seen by bfp_vec_from_f64
 *   slots 16..287 are the library's reduction scratch (a ticket counter and
 *   sixteen accumulator sets on separate cache lines); bfp_vec_init (or
 *   bfp_meta_reset) must prepare them once, and every operation leaves them
 *   prepared again. */
#define BFP_META_SLOTS 288
#define BFP_META_EXP 0
#define BFP_META_MAX 1
#define BFP_META_MIN 2
#define BFP_META_SAT 3
#define BFP_META_MU 4
#define BFP_META_FLAGS 5

/* One BFP block on a padded vertex-centred grid (D1 of Section 2: one
 * exponent for the whole block). The grid has n interior points per
 * dimension and a ring of Dirichlet boundary points that always holds zero
 * mantissas: (n+2)^ndim points, x fastest. Storage is row-pitched: the
 * (n+2)^(ndim-1) rows (y, or z-then-y) each hold `pitch` elements, of which
 * the first n+2 are the grid row and the rest are zero padding. Use
 * bfp_layout() for pitch and size. */
typedef struct {
  void* mant;           /* device, int8/int16/int32 per storage_bits        */
  int64_t* meta;        /* device, BFP_META_SLOTS int64                      */
  int32_t w;            /* mantissa width, 1 <= w <= storage_bits            */
  int32_t storage_bits; /* 8, 16 or 32                                       */
  int32_t ndim;         /* 2 or 3                                            */
  int32_t n;            /* interior points per dimension (>= 1)              */
  int64_t pitch;        /* elements per row, from bfp_layout                 */
} bfp_vec;

/* A BFP scalar (block of size one): value m * 2^exp, |m| < 2^(w-1). */
typedef struct {
  int64_t m;
  int64_t exp;
  int32_t w;
} bfp_scalar;

/* A constant-coefficient BFP matrix on padded grids (a sparse matrix with
 * one shared exponent, D9): tap mantissas at offsets o in {-1,0,1}^ndim,
 * index ((oz+1)*3 + (oy+1))*3 + (ox+1) (2D: (oy+1)*3 + (ox+1)).
 *   BFP_STENCIL_A  same grid:       z[p] = sum_o t[o] x[p + o]
 *   BFP_STENCIL_R  fine -> coarse:  z[I] = sum_o t[o] x[2I + o]
 *   BFP_STENCIL_P  coarse -> fine:  z[p] = sum_o t[o] u[p + o], u the coarse
 *                  block placed on the even fine nodes, zero elsewhere.
 * Only interior output points are computed; the output ring stays zero. */
typedef enum { BFP_STENCIL_A = 0, BFP_STENCIL_R = 1, BFP_STENCIL_P = 2 } bfp_stencil_kind;
typedef struct {
  int32_t ndim;
  int32_t kind;
  int64_t exp;
  int32_t w;            /* max msb of the taps (bound used by width checks) */
  int32_t taps[27];
} bfp_stencil;

/* The estimate gamma >= ||z||_inf needed by BFP_SATURATE (Table 1). Only
 * floor(log2 gamma) matters. Norms are read from device metadata, so the
 * estimate is evaluated on the device when the operation runs.
 *   BFP_GAMMA_NORM     gamma = c * ||a||_inf           (c > 0)
 *   BFP_GAMMA_SUM      gamma = ||a||_inf + ||b||_inf
 *   BFP_GAMMA_EXPLICIT gamma = c                        (c >= 0)        */
typedef enum { BFP_GAMMA_NORM = 1, BFP_GAMMA_SUM = 2, BFP_GAMMA_EXPLICIT = 3 } bfp_gamma_rule;
typedef struct {
  int32_t rule;
  const int64_t* a_meta; /* device meta of the block in the first norm     */
  const int64_t* b_meta; /* device meta of the block in the second norm    */
  bfp_scalar c;          /* multiplier (NORM) or value (EXPLICIT), |m| < 2^24 */
} bfp_gamma;

/* ------------------------------------------------------------ layout --- */

/* Row pitch (elements, a multiple of 128 bytes: rows start on cache-line
 * boundaries when the block is 128-byte aligned) and byte size of a block.
 * Blocks laid out by hand need only a pitch that is a multiple of 16 bytes
 * and holds n + 2 elements, and 16-byte aligned mantissas.               */
int bfp_layout(int ndim, int n, int storage_bits, int64_t* pitch, size_t* bytes);

/* Make v the zero block: all mantissas (ring and padding included) 0,
 * e = 1 - w, MAX = MIN = 0, counters and reduction scratch reset.        */
int bfp_vec_init(const bfp_vec* v, void* stream);

/* Declare that v's mantissas, written by the caller (each in X_w, ring and
 * padding zero), carry the exponent `exp`: sets e and recomputes MAX / MIN
 * on the device. The mantissas are left unchanged.                        */
int bfp_vec_assign(bfp_vec* v, int64_t exp, void* stream);

/* Reset only the metadata reduction scratch of `meta` (after the caller
 * filled the slots some other way).                                      */
int bfp_meta_reset(int64_t* meta_dev, void* stream);

/* ---------------------------------------------------------- a1: quant --- */

/* dst = Q_w(src * 2^log2_scale): normalized floor quantization of exact FP64
 * values (the `quant` steps of IR, V and FMG; rounding = floor as for every
 * truncation in Section 2): e = max_i nu(x_i) - w, m_i = floor(x_i / 2^e),
 * where nu(q) is the smallest b with -2^(b-1) <= q < 2^(b-1). An all-zero
 * input gets e = 1 - w + log2_scale. src_dev is dense (n+2)^ndim FP64 in
 * x-fastest order; ring values are ignored (the ring stays zero). A NaN or
 * Inf sets bit 0 of meta[BFP_META_FLAGS]; bfp_vec_check reports it. Two
 * launches (a max-reduction, then the conversion).                        */
int bfp_vec_from_f64(const double* src_dev, int64_t log2_scale, bfp_vec* dst, void* stream);

/* dst_dev (dense (n+2)^ndim FP64) = m * 2^e; exact for w <= 53 whenever the
 * results are normal doubles.                                             */
int bfp_vec_to_f64(const bfp_vec* src, double* dst_dev, void* stream);

/* Synchronizes `stream`; BFP_ENONFINITE if v's non-finite flag is set.    */
int bfp_vec_check(const bfp_vec* v, void* stream);

/* ------------------------------------------- a2-a4: gemv and special cases */

/* z = alpha * A x + beta * y (gemv, equation (4.1) of Section 4, computed by
 * the exact gemv setup/row of Appendix B and quantized by `mode`); with
 * y == NULL it is the exact SpMV z = alpha * A x (espmv). A is a stencil
 * (A, R or P); x must be on A's input grid, y and z on its output grid.
 * Exact intermediates: |alpha_m| * sum|taps| * 2^(w_x-1) and
 * |beta_m| * 2^(w_y-1) must stay below 2^61 (else BFP_EWIDTH). z may alias
 * y but not x. gamma is read only in BFP_SATURATE mode.                   */
int bfp_stencil_apply(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                      const bfp_scalar* beta, const bfp_vec* y, int w_out, int mode,
                      const bfp_gamma* gamma, bfp_vec* z, void* stream);

/* r = A x - b (the IR and V-cycle residuals of Appendix C).               */
int bfp_residual(const bfp_stencil* A, const bfp_vec* x, const bfp_vec* b, int w_out,
                 int mode, const bfp_gamma* gamma, bfp_vec* r, void* stream);

/* z = alpha * x + beta * y (exact axpby setup/row, Appendix B). z may alias
 * x or y.                                                                 */
int bfp_axpy(const bfp_scalar* alpha, const bfp_vec* x, const bfp_scalar* beta,
             const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma, bfp_vec* z,
             void* stream);

/* z = x - y aligned at min(e_x, e_y) (the qsub of IR, Appendix C).          */
int bfp_sub(const bfp_vec* x, const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma,
            bfp_vec* z, void* stream);

/* ---------------------------------------------------------- a5: dot ----- */

/* Exact dot product sum_i x_m,i * y_m,i (Section 2 remark on BFP dot
 * products: no alignment shifts, exponent e_x + e_y, accumulator growing
 * with log2 n). out_dev: BFP_META_SLOTS int64, of which [0] = low and
 * [1] = high 64 bits of the two's-complement 128-bit mantissa, [2] =
 * exponent; [16..] are the library's reduction scratch and must be zero
 * before the first call (they are left zero after every call).            */
int bfp_dot(const bfp_vec* x, const bfp_vec* y, int64_t* out_dev, void* stream);

/* Plain device copy of `bytes` from src_dev to dst_dev (both 16-byte
 * aligned, bytes a multiple of 16; the ranges must not overlap) with
 * 16-byte loads and stores, grid-strided, "stream_copy_per_thread" (4 or
 * 8, default 4) words in flight per thread on at most
 * "stream_copy_blocks" (default 1024) workgroups (nontemporal = 1:
 * non-temporal loads and stores). Not a BFP operation: the streaming-
 * bandwidth reference that the roofline fractions of the BFP kernels are
 * read against. Asynchronous on `stream`. BFP_EINVAL on a bad size,
 * alignment or NULL pointer (bytes = 0: nothing to do).                   */
int bfp_stream_copy(const void* src_dev, void* dst_dev, int64_t bytes, int nontemporal,
                    void* stream);

/* ------------------------------------------------ a7, a8: requantization */

/* out = qcomp of the copy of in to w_out bits (normalized, floor): one pass,
 * mu* comes from in's MAX / MIN metadata. out may alias in.              */
int bfp_normalize(const bfp_vec* in, int w_out, bfp_vec* out, void* stream);

/* out = nnqcomp of the copy of in: exponent from gamma, floor shift,
 * saturation to X_w_out (Algorithm 3). out may alias in.                 */
int bfp_saturate_truncate(const bfp_vec* in, int w_out, const bfp_gamma* gamma, bfp_vec* out,
                          void* stream);

/* ------------------------------------------------------ multigrid ------ */

/* Exact Chebyshev coefficients (algorithm "Coefficients for two Chebyshev
 * iterations", Appendix C) for rho = rho_num/rho_den and eta =
 * eta_num/eta_den, multiplied by (scale_num/scale_den) for c1 and its square
 * for c2 (the rescaling to a stored operator whose diagonal is
 * scale_den/scale_num), each floor-quantized normalized to w bits.       */
int bfp_cheby_coeffs(int64_t rho_num, int64_t rho_den, int64_t eta_num, int64_t eta_den,
                     int64_t scale_num, int64_t scale_den, int w, bfp_scalar* c1,
                     bfp_scalar* c2);

/* Quantization policy of the solver: which calls use BFP_NORMALIZE.        */
typedef enum {
  MG_POLICY_Q = 0,              /* every call qcomp                          */
  MG_POLICY_NN = 1,             /* every call nnqcomp (Section 6.4)          */
  MG_POLICY_NN_IR_FIRST_Q = 2,  /* qcomp for the first IR residual per level */
  MG_POLICY_NN_IR_FIRST2_Q = 3, /* ... and the first two of a plain IR solve */
  MG_POLICY_NN_IR_Q = 4         /* qcomp for every IR residual               */
} mg_policy;

#define MG_MAX_LEVELS 16

/* Problem and schedule of one solve: -Laplace u = f on the unit square
 * (ndim 2, 5-point) or cube (ndim 3, 7-point), homogeneous Dirichlet,
 * levels 1..L with n_j = 2^j - 1. Widths are indexed by level j (entry 0
 * unused): w_check for A and b, w_work for the iterate x, w_inner for the
 * V-cycle (the three precisions of Section 5).                            */
typedef struct {
  int32_t ndim, L;
  int32_t nu1, nu2;   /* V(nu1, nu2); nu1 >= 1. The paper's cycle is V(1,0) */
  int32_t N;          /* IR-V iterations per FMG level                     */
  int32_t policy;     /* mg_policy                                          */
  int32_t min_storage_bits; /* 0, 8, 16 or 32: smallest storage for any block;
                         otherwise the narrowest type holding the width   */
  int32_t w_check[MG_MAX_LEVELS + 1];
  int32_t w_work[MG_MAX_LEVELS + 1];
  int32_t w_inner[MG_MAX_LEVELS + 1];
  bfp_scalar c1, c2;  /* relaxation y = c2 A r + c1 r for the stored A       */
  bfp_scalar c1_gamma;/* c1 of D^-1 A, used in the V-residual estimate       */
} mg_params;

/* Fill *out with a complete schedule for -Laplace u = f on levels 1..L:
 *   progressive = 0: every width (check, work, inner) equals w;
 *   progressive = 1: check 32, working w_j = min(32, 2j + 8) and inner
 *     w_j = min(working, max(5, w - (L - j))) (widths grow linearly with the
 *     level, eq. width-bounds of Section 5, with m = 1 for Poisson; w is the
 *     finest inner width);
 * and Chebyshev coefficients for rho = 2 (an upper bound of the spectrum of
 * D^-1 A on every level) and eta = eta_percent / 100, rescaled to the stored
 * operator (diag 1 in 2D, 3/4 in 3D) and floor-quantized to 16 bits.      */
int mg_params_init(int ndim, int L, int w, int progressive, int nu1, int nu2, int N,
                   int policy, int eta_percent, mg_params* out);

/* ---- A priori precision estimation (Section 6.2) and eta (Section 5) ----
 * Host-driven set-up computations on a coarse estimation level j = prm->L
 * (at most 7 in 2D, 5 in 3D). They run many device solves and synchronize
 * with the host; they are not steps of a solve.                          */

/* rho_v = ||E||_A for E (host, N x N doubles, column k = E e_k, interior
 * points ordered x fastest, N = (2^j - 1)^ndim) and the scaled 5- or
 * 7-point operator A of level j: the square root of the largest
 * generalized eigenvalue of E^T A E x = lambda A x (conv-rate-v-cycle of
 * Section 6.2; scaling A does not change it).                            */
int bfp_energy_norm(const double* E, int ndim, int j, double* rho);

/* Device bytes mg_error_propagation / mg_conv_rate / mg_prec_est /
 * mg_eta_scan need in their arena for the schedule prm (0 on error).     */
size_t mg_conv_rate_bytes(const mg_params* prm);

/* E of one IR-V iteration (mg_ir with iters = 1, b = 0) on level prm->L,
 * built on the device from the canonical basis vectors e_k quantized at
 * w_work[L] (mantissa 2^(w-2), exponent 2 - w); E_host receives N x N
 * doubles, column by column. Uses and overwrites the arena; synchronizes
 * `stream`.                                                               */
int mg_error_propagation(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                         double* E_host);

/* conv-rate-v-cycle: bfp_energy_norm of mg_error_propagation's E.        */
int mg_conv_rate(const mg_params* prm, void* arena_dev, size_t bytes, void* stream, double* rho);

/* The width rules of Algorithm bfp-prec-est applied to p (levels 1..p->L):
 * check w_j = j (m + k) + q_check and inner w_j = j m + q_inner (2m = the
 * order of the PDE, k = the approximation order; 1 and 2 for the FD
 * Poisson problems), capped at 32 bits, the check width raised to at least
 * and the inner width lowered to at most the working width p->w_work[j],
 * which is kept.                                                         */
int mg_params_apply_estimate(mg_params* p, int q_check, int q_inner, int m, int k);

typedef struct {
  int32_t q_check, q_inner; /* constants of the check and inner width rules */
  double rho_ref;           /* rate with both constants at q_max            */
  double rho;               /* rate with (q_check, q_inner)                 */
  int32_t rates;            /* distinct width schedules evaluated           */
} mg_prec_est_result;

/* Algorithm bfp-prec-est on level j_c = base->L: q_check is the smallest q
 * in 1..q_max (binary search) whose rate, with the inner constant at q_max,
 * is below rho_thresh times the reference rate; q_inner the smallest with
 * the check constant q_check. base supplies everything else (working
 * widths, cycle, policy, Chebyshev coefficients).                        */
int mg_prec_est(const mg_params* base, int q_max, double rho_thresh, int m, int k,
                void* arena_dev, size_t bytes, void* stream, mg_prec_est_result* out);

/* The Chebyshev parameter eta = i / 100, i in lo..hi (1 <= lo <= hi <= 99),
 * with the smallest rate rho_v on level base->L (the minimization of
 * Section 5, every i evaluated, ties to the smaller i); rates (optional,
 * hi - lo + 1 doubles) receives every rate.                              */
int mg_eta_scan(const mg_params* base, int lo, int hi, void* arena_dev, size_t bytes,
                void* stream, int* eta_percent, double* rho, double* rates);

typedef struct mg_hierarchy mg_hierarchy;

/* Device bytes a hierarchy needs in its arena.                            */
size_t mg_hierarchy_bytes(const mg_params* prm);

/* Carve a hierarchy out of a caller-provided device arena (at least
 * mg_hierarchy_bytes, 256-byte aligned) and zero it on `stream`. The
 * hierarchy object itself lives in host memory; destroy it with
 * mg_hierarchy_destroy (the arena stays the caller's).                    */
int mg_hierarchy_create(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                        mg_hierarchy** out);
int mg_hierarchy_destroy(mg_hierarchy* h);

/* b_j = quant(f_j / s_j) at w_check[j]: f_dev holds FP64 samples of f on the
 * padded level-j grid (dense (n_j+2)^ndim); s_j = 4/h^2 in 2D, 8/h^2 in 3D
 * (the scaling of setup S; a power of two, applied exactly).            */
int mg_set_rhs(mg_hierarchy* h, int level, const double* f_dev, void* stream);

/* x_level = quant(x0) at w_work[level] (an initial guess for mg_ir).     */
int mg_set_x(mg_hierarchy* h, int level, const double* x0_dev, void* stream);

/* FMG (Appendix C): x_1 = 0, then per level l = 1..L: x_l = P x_(l-1) (l>1)
 * and N IR-V(nu1,nu2) iterations. Result in the level-L iterate.          */
int mg_fmg(mg_hierarchy* h, void* stream);

/* One whole solve from FP64 data: mg_set_rhs for every level j = 1..L with
 * f_dev = rhs_dev[j-1] (a host array of L device pointers), then mg_fmg;
 * results are identical to those calls. The levels the coarse-level program
 * runs are quantized inside that program, and the finer levels on a second
 * stream owned by the hierarchy (created on the first call, default
 * priority) while the program runs; that stream starts after the work
 * issued on `stream` so far, and `stream` waits for it before the finer
 * levels' FMG, so the call is ordered on `stream` like the others.
 * The second stream lives as long as the hierarchy and, like any HIP
 * stream, takes one of the process's hardware queues (GPU_MAX_HW_QUEUES):
 * destroy hierarchies that are done with to leave queues to other streams.
 * rhs_dev is read during the call only. Errors: BFP_EINVAL for a NULL
 * argument or level pointer (nothing issued), BFP_EHIP if the stream or
 * events cannot be created.                                              */
int mg_fmg_f64(mg_hierarchy* h, const double* const* rhs_dev, void* stream);

/* IR-V with the safety mechanism of Section 6.4 (a solver that skips
 * normalization watches its residual and runs Algorithm 1 — qcomp — for
 * some operations during some iterations when convergence stalls): like
 * mg_ir, except that after an iteration whose IR residual saturated any
 * entry (the nnqcomp estimate was too small) or whose residual norm exceeds
 * theta = theta_num / 2^theta_log2den times the previous one, the IR
 * residuals of the next q_iters iterations use qcomp. The norms and the
 * saturation count are read after every iteration, so the call synchronizes
 * `stream` once per iteration. *switched (nullable) receives the number of
 * iterations that ran the fallback. BFP_EINVAL for a bad level, iters < 0,
 * q_iters < 0, theta_num < 1 or theta_log2den outside [0, 62].           */
int mg_ir_safe(mg_hierarchy* h, int level, int iters, int q_iters, int32_t theta_num,
               int32_t theta_log2den, int* switched, void* stream);

/* Diagnostics of the solves run on a hierarchy (Section 4's qcomp window,
 * Table 2, and nnqcomp saturation, Section 6.4), kept on the device by every
 * quantizing call the mg_* functions issue, counted per recursion level
 * (the level of the call's input for a restriction, of its output
 * otherwise) and call site:
 *   sites: 0 IR residual (first iteration), 1 IR residual (later), 2 IR
 *   correction, 3 relaxation, 4 V-cycle residual, 5 restriction, 6 V-cycle
 *   correction, 7 FMG prolongation.
 *   bins, MG_DIAG_BINS per (level, site):
 *     0 .. MG_DIAG_GAP_BINS-1: qcomp calls that have an estimate gamma, by
 *       the window gap d = mu_tmp - mu* (mu_tmp = nu(gamma) - e_z*, mu* the
 *       exact result's leading bit): bin 0 for d < 0, bin 1 + min(d, 59).
 *       Algorithm 1 with w_tmp = w_out + w_add recomputes exactly the calls
 *       with d < 0 (overflow) or d > w_add (underflow);
 *     61: nnqcomp calls; 62: entries they saturated; 63: nnqcomp calls that
 *       saturated at least one entry.
 * mg_diag_read synchronizes `stream`, copies the counters to host_out
 * (int64, [MG_MAX_LEVELS + 1][MG_DIAG_SITES][MG_DIAG_BINS], row 0 unused)
 * and, when reset != 0, zeroes them. Counters start at zero when the
 * hierarchy is created. Only hierarchies created with the tuning key
 * "diagnostics" set keep them (each diagnosed call ends with a few
 * device-scope atomic adds, which cost a few percent of a solve).
 * BFP_EINVAL for a NULL argument or a hierarchy without diagnostics. Work
 * still running on other streams is not waited for.                      */
#define MG_DIAG_SITES 8
#define MG_DIAG_BINS 64
#define MG_DIAG_GAP_BINS 61
int mg_diag_read(mg_hierarchy* h, int64_t* host_out, int reset, void* stream);

/* `iters` IR-V(nu1,nu2) iterations on level `level` from its current x.   */
int mg_ir(mg_hierarchy* h, int level, int iters, void* stream);

/* y = V(r) on `level` (r, y on the level-`level` grid at w_inner[level]).  */
int mg_vcycle(mg_hierarchy* h, int level, const bfp_vec* r, bfp_vec* y, void* stream);

/* Views of the hierarchy's blocks (device pointers into the arena).
 * which: 0 = x (iterate), 1 = b (right-hand side), 2 = r (last IR residual). */
int mg_get_vec(mg_hierarchy* h, int level, int which, bfp_vec* out);

/* Per-level algorithmic byte counts of everything enqueued so far, and
 * the number of kernel launches (host-side counters).                     */
int mg_counters(const mg_hierarchy* h, double* bytes, int64_t* launches);

/* ---------------------------------------------------------- batches ---
 * Many independent problems solved together (the batched workload): each
 * problem has its own hierarchy inside one caller-provided arena, and
 * mg_solve_batch runs, for every problem, the FP64 -> BFP conversion of its
 * right-hand side on every level followed by the whole FMG of mg_fmg, in ONE
 * launch (one workgroup per problem, larger problems first). Results are
 * bit-identical to solving each problem alone with mg_set_rhs + mg_fmg.
 * prms[i]: the parameters of problem i (all with the same ndim, 2^L - 1 <
 * 1024 points per dimension); problems with bitwise-identical parameters
 * share one recorded program. Creation synchronizes `stream`.             */
typedef struct mg_batch mg_batch;

size_t mg_batch_bytes(const mg_params* prms, int nprob);      /* 0 on error */
int mg_batch_create(const mg_params* prms, int nprob, void* arena_dev, size_t bytes,
                    void* stream, mg_batch** out);
int mg_batch_destroy(mg_batch* b);

/* rhs_table_dev: device array of nprob * MG_MAX_LEVELS FP64 pointers; entry
 * [i * MG_MAX_LEVELS + j - 1] is problem i's f_j on its padded level-j grid
 * ((2^j + 1)^ndim values; ring ignored), as for mg_set_rhs.               */
int mg_solve_batch(mg_batch* b, const double* const* rhs_table_dev, void* stream);

/* Views of problem `prob`'s blocks (which as for mg_get_vec).              */
int mg_batch_get_vec(mg_batch* b, int prob, int level, int which, bfp_vec* out);

/* Algorithmic bytes of one mg_solve_batch and the launches issued so far.  */
int mg_batch_counters(const mg_batch* b, double* bytes, int64_t* launches);

/* ---------------------------------------------------------- serving ---
 * A request server (the serving workload): independent solves of mixed
 * dimensions, sizes and widths are submitted without blocking and run
 * concurrently in up to max_slots execution slots (one HIP stream each,
 * default priority). Each request needs a resident hierarchy for its
 * parameters inside the caller's arena (the HBM budget): hierarchies are
 * reused across requests with bitwise-identical parameters, created while
 * the budget allows and evicted least-recently-used when idle; a request
 * waits while neither a slot nor memory is free (admission in arrival
 * order). A slot runs the whole solve: mg_set_rhs on every level, mg_fmg,
 * and the finest iterate converted to FP64 into x_out_dev. Results are
 * bit-identical to the same solve run alone. The slots' streams do not wait
 * on any other stream: a request's buffers must be ready (the work that
 * fills them finished) when it is submitted. Hierarchy creation on first
 * use of a parameter set synchronizes that slot's stream. Not thread-safe:
 * one host thread drives a server. Slots overlap only as far as the HIP
 * runtime has hardware queues: set GPU_MAX_HW_QUEUES (HIP's default is 4)
 * before the process initializes HIP; 16 queues with 16 slots measured
 * best on MI355X.                                                        */
typedef struct mg_server mg_server;
typedef struct {
  int32_t max_slots;   /* requests on the device at once, 1..64            */
  int32_t max_queue;   /* queued requests beyond which submit is BFP_EBUSY  */
  int32_t exec_max_points; /* levels with at most this many points run in
                              the one-workgroup recorded programs of the
                              server's hierarchies; 0 = 70000 (2D up to
                              255^2, 3D up to 31^3)                        */
} mg_server_cfg;
typedef struct {
  mg_params prm;                          /* shape, widths, schedule       */
  const double* rhs_dev[MG_MAX_LEVELS];   /* [j-1]: FP64 f_j on the padded
                                             level-j grid (device); must stay
                                             valid until the request is done */
  double* x_out_dev;                      /* (2^L + 1)^ndim FP64 values     */
} mg_request;
typedef struct {
  int32_t status;      /* BFP_OK or the error that ended the request        */
  float gpu_ms;        /* device time from the request's first to last op   */
} mg_result;

int mg_server_create(const mg_server_cfg* cfg, void* arena_dev, size_t bytes, mg_server** out);
/* Queue a request (non-blocking); BFP_EBUSY when the queue is full.       */
int mg_server_submit(mg_server* s, const mg_request* req, uint64_t* ticket);
/* Make progress (retire finished slots, admit queued requests) and report
 * on `ticket`: BFP_OK (result in *out, ticket released), BFP_PENDING, or an
 * error. Never blocks.                                                    */
int mg_server_poll(mg_server* s, uint64_t ticket, mg_result* out);
/* Make progress and hand over up to `cap` finished requests (tickets and
 * results, in no particular order; their tickets are released); *count is
 * the number handed over. Never blocks.                                   */
int mg_server_collect(mg_server* s, uint64_t* tickets, mg_result* results, int cap, int* count);
int mg_server_stats(const mg_server* s, int* queued, int* running, size_t* resident_bytes);
int mg_server_destroy(mg_server* s);

/* ---- Solve without device allocation ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): mg_fmg_f64 (FMG from the FP64 right-hand
 * sides rhs_dev[j-1] of levels j = 1..prm->L, as for mg_fmg_f64) on a
 * hierarchy the library keeps in a static device array of MG_NOALLOC_BYTES
 * per GPU (held until the process ends), then x_out_dev (dense
 * (n_L + 2)^ndim doubles) = the finest iterate (exact for working widths
 * up to 53 bits). Problems whose hierarchy needs more than MG_NOALLOC_BYTES
 * (mg_hierarchy_bytes; 2D up to 513^2, 3D up to 65^3 fit) are rejected with
 * BFP_ENOMEM. The first call for a parameter set on a device lays the
 * hierarchy out in the array (host work and one synchronization of
 * `stream`); later calls with the same parameters only enqueue the solve
 * on `stream`. No hipMalloc / hipFree is called. Every call on a GPU uses
 * that GPU's one array, which keeps the last call's contents: calls that
 * overlap in time on one GPU (different streams or host threads without
 * ordering) race and must be serialized by the caller.                   */
#define MG_NOALLOC_BYTES (32u << 20)
int mg_fmg_f64_noalloc(const mg_params* prm, const double* const* rhs_dev, double* x_out_dev,
                       void* stream);

/* ---- FP64 multigrid comparator ----
 * The same FMG schedule as the BFP solver (x_1 = 0, FMG prolongation, N
 * IR-V(nu1, nu2) iterations per level, relaxation y = c2 A r + c1 r, the
 * V-cycle of Appendix C with its added sweeps) on the same scaled operators,
 * in IEEE double arithmetic on the GPU: the floating-point multigrid the
 * BFP solves are compared with. c1, c2 are the coefficients for the stored
 * operator (the doubles of mg_params.c1 / c2). Levels are dense padded
 * FP64 grids in the caller's arena (fp64_mg_bytes).                      */
typedef struct fp64_mg fp64_mg;
size_t fp64_mg_bytes(int ndim, int L);   /* 0 on error */
int fp64_mg_create(int ndim, int L, int nu1, int nu2, int N, double c1, double c2, void* arena_dev,
                   size_t bytes, void* stream, fp64_mg** out);
/* rhs_dev[j-1]: f_j on the padded level-j grid (as for mg_set_rhs);
 * x_out_dev: dense (n_L + 2)^ndim doubles, the FMG solution.             */
int fp64_mg_fmg(fp64_mg* h, const double* const* rhs_dev, double* x_out_dev, void* stream);
int fp64_mg_destroy(fp64_mg* h);

/* ---- Sub-maximal block sizes (Section 2, Remark "Block size") ----
 * A tiled BFP grid vector: the interior points of every grid row (fastest
 * axis x) are split into tiles of T consecutive points (T a power of two in
 * 1..256; the last tile of a row holds n mod T points when T does not
 * divide n), and every tile is a BFP block of its own: one exponent and
 * w-bit mantissas. Block size 1 is floating point with a w-bit significand
 * rounded toward minus infinity; the rest of this library is the maximal
 * block (one exponent per vector).
 *   mant  device, the padded (n+2)^ndim grid (x fastest, row pitch `pitch`
 *         elements from bfp_tiles_layout), int8/int16/int32 by
 *         storage_bits; the ring is zero and no operation writes it.
 *   exps  device, one int32 exponent per tile: n^(ndim-1) rows of ceil(n/T)
 *         tiles, row r = (z-1) n + (y-1) in 3D and y - 1 in 2D (padded
 *         coordinates), tile t holding x = t T + 1 .. min((t+1) T, n).
 * Both arrays are caller-owned. Exponents must stay within +-2^30.
 *
 * Every operation computes each interior point's exact value and quantizes
 * every output tile on its own to z->w bits with the normalized floor
 * quantization of Section 2 (what Algorithm 1 returns, per tile): e = the
 * largest nu over the tile's nonzero values minus w, m_i = floor(v_i / 2^e);
 * an all-zero tile gets e = 1 - w. One pass, no reduction beyond a tile.
 * Exact range: the terms of one point (for the stencil, alpha times a tap
 * times a neighbour at exponent alpha.exp + A->exp + the neighbour's tile
 * exponent, and beta y at beta.exp + y's tile exponent) are summed exactly
 * while their exponents lie within 60 of each other; a point spread wider
 * is set to zero and counted into *status_dev (device int32, added to, not
 * reset; NULL: not counted). Coefficient limits: |alpha.m|, |beta.m| <
 * 2^16, |taps| < 2^15 (else BFP_EWIDTH). Operands must share ndim, n and T
 * (else BFP_ESHAPE). All calls are asynchronous on `stream`.             */
typedef struct {
  void* mant;
  int32_t* exps;
  int32_t w;            /* mantissa width, 1 <= w <= storage_bits            */
  int32_t storage_bits; /* 8, 16 or 32                                       */
  int32_t ndim;         /* 2 or 3                                            */
  int32_t n;            /* interior points per dimension                     */
  int32_t T;            /* tile size                                         */
  int64_t pitch;        /* elements per row                                  */
} bfp_tiles;
/* Row pitch, mantissa bytes and exponent bytes of a tiled vector.        */
int bfp_tiles_layout(int ndim, int n, int T, int storage_bits, int64_t* pitch, size_t* mant_bytes,
                     size_t* exp_bytes);
/* Zero mantissas (ring included) and every tile exponent 1 - w.          */
int bfp_tiles_init(const bfp_tiles* t, void* stream);
/* quant of FP64 data, tile by tile: x_dev is the padded (n+2)^ndim grid
 * (contiguous, ring not read); non-finite values become 0 and are counted
 * into *status_dev.                                                      */
int bfp_tiles_from_f64(const double* x_dev, bfp_tiles* out, int32_t* status_dev, void* stream);
/* m 2^e into the interior points of the padded (n+2)^ndim FP64 grid x_dev
 * (ring untouched); exact while the values are normal or subnormal
 * doubles.                                                               */
int bfp_tiles_to_f64(const bfp_tiles* in, double* x_dev, void* stream);
/* z = alpha A x + beta y (y may be NULL: z = alpha A x), A a same-grid star
 * stencil (BFP_STENCIL_A with nonzero taps only at the centre and the 2 ndim
 * axis neighbours; else BFP_EINVAL), the exact gemv row of Appendix B per
 * point with the operand tiles' exponents. z must not alias x (y may).    */
int bfp_tiles_stencil_apply(const bfp_stencil* A, const bfp_tiles* x, const bfp_scalar* alpha,
                            const bfp_scalar* beta, const bfp_tiles* y, bfp_tiles* z,
                            int32_t* status_dev, void* stream);
/* z = alpha x + beta y point by point (the exact axpby row of Appendix B
 * with each point's tile exponents); z may alias x or y.                 */
int bfp_tiles_axpby(const bfp_scalar* alpha, const bfp_tiles* x, const bfp_scalar* beta,
                    const bfp_tiles* y, bfp_tiles* z, int32_t* status_dev, void* stream);

/* ---- The paper's finite-element model problems (Section 6) ----
 * 1D Rayleigh-Ritz B-spline discretizations of Poisson (m = 1) and the
 * biharmonic equation (m = 2) with strongly imposed Dirichlet conditions,
 * solved by BFP FMG (Appendix C: FMG with N IR-V(1,0) iterations per
 * level). The caller supplies the problem: per level j = 1..L the reference
 * stiffness matrix K_hat_j (unit mesh spacing; K_j = h^(1-2m) K_hat_j), for
 * j >= 2 the prolongation P_j from level j-1 (fine rows, coarse columns),
 * both as banded matrices of exact rationals, and the FP64 load vector
 * F_hat_j (F_j = h F_hat_j). The library applies Set-up S exactly
 * (A_j = D_j^-1 K_j, b_j = D_j^-1 F_j, R_j = D_(j-1)^-1 P_j^T D_j, 128-bit
 * rational arithmetic; BFP_EWIDTH if a value does not fit) and quantizes
 * each operator per call site (A at w_check for the IR residual, A, R, P at
 * w_inner inside the V-cycle, P at w_work for the FMG prolongation: Q_w of
 * the whole matrix, one exponent). Chebyshev c1, c2 come from the
 * Gershgorin bound of A on level min(5, L) and eta = eta_num / eta_den,
 * floor-quantized to 16 bits. Every operation is a qcomp. Blocks are int32
 * with 61-bit exact budgets: an operation whose terms could exceed them
 * fails with BFP_EWIDTH (keep w_check + w_work and 16 + w_inner + the
 * inner-width tap bits within 61). The hierarchy allocates its own device
 * memory (hipMalloc at creation, freed by fe_hierarchy_destroy).        */
typedef struct {
  int32_t nrows, ncols;
  int32_t band;            /* entries stored per row                        */
  const int32_t* col0;     /* host: first column of each row                */
  const int64_t* num;      /* host: nrows x band numerators                 */
  const int64_t* den;      /* host: nrows x band denominators (> 0)         */
} fe_rational_band;
typedef struct {
  int32_t m;               /* 1: Poisson, 2: biharmonic                     */
  int32_t L, N;            /* levels; IR-V iterations per FMG level         */
  int32_t eta_num, eta_den;
  int32_t w_check[MG_MAX_LEVELS + 1], w_work[MG_MAX_LEVELS + 1],
      w_inner[MG_MAX_LEVELS + 1];
} fe_params;
typedef struct fe_hierarchy fe_hierarchy;
/* K[j-1], P[j-1] (P[0] unused), F[j-1]: level j. Synchronizes. When every
 * block has at most 4096 unknowns the hierarchy also records its whole FMG
 * as one program (a device array of op descriptors) for fe_fmg.          */
int fe_hierarchy_create(const fe_params* prm, const fe_rational_band* K, const fe_rational_band* P,
                        const double* const* F, void* stream, fe_hierarchy** out);
/* FMG from x_1 = 0; the solution is block x of level L. Asynchronous: one
 * single-workgroup launch of the recorded program (tuning key
 * "fe_program"), else one launch per operation.                          */
int fe_fmg(fe_hierarchy* h, void* stream);
/* Copy block `which` (0 x, 1 b, 2 the last IR residual) of a level to the
 * host: n + 2 int32 mantissas (the two ends zero) into mant_host (may be
 * NULL), its exponent, its n. Synchronizes the device.                    */
int fe_get(fe_hierarchy* h, int level, int which, int32_t* mant_host, int64_t* exp_out, int* n_out);
/* The quantized Chebyshev coefficients the hierarchy uses.               */
int fe_coefficients(const fe_hierarchy* h, bfp_scalar* c1, bfp_scalar* c2);
/* Bytes the operations moved and kernel launches, since creation.         */
int fe_counters(const fe_hierarchy* h, double* bytes, int64_t* launches);
int fe_hierarchy_destroy(fe_hierarchy* h);

/* Launch-shape autotuning for the levels of h above its coarse-level
 * executor: per level j, every march length of the star kernel (rows or
 * planes per wave, 1..64) on the IR residual r = A x - b, and of the
 * transfer kernels (coarse rows or planes per wave, 1..32) on the
 * restriction into level j - 1 plus the prolongation-correction from it,
 * is timed on `stream` with HIP events (median of three runs of `reps`
 * back-to-back launches on h's own blocks); the fastest, when it beats the
 * default shape, is kept in the process-wide per-level table that every
 * later launch on grids of that size uses (an explicit tuning key still
 * takes precedence). Results never depend on launch shapes. Overwrites h's
 * work blocks (r, s, t, the restricted residuals): set the right-hand side
 * again before solving. Synchronizes `stream`. out (nullable) receives the
 * chosen shapes (0 = default kept) and the times.                        */
typedef struct {
  int32_t first_level, last_level;
  int32_t star_rows[MG_MAX_LEVELS + 1], transfer_rows[MG_MAX_LEVELS + 1];
  float star_us[MG_MAX_LEVELS + 1], star_default_us[MG_MAX_LEVELS + 1];
  float transfer_us[MG_MAX_LEVELS + 1], transfer_default_us[MG_MAX_LEVELS + 1];
} mg_tune_report;
int mg_autotune(mg_hierarchy* h, int reps, void* stream, mg_tune_report* out);
/* The same per-level shapes chosen by the time of whole FMG solves
 * (mg_fmg on h's current right-hand sides): from the finest level down,
 * each level's star march length (1..64) and then its transfer march
 * length (1..32) is timed in turns with the incumbent (first the default
 * shape; three runs of `reps` solves each, medians compared, so a clock
 * drift during the search favours neither) with every other level at its
 * current shape; a candidate replaces the incumbent when at least 0.3%
 * faster. Every shape is so judged in the solve's own conditions (caches,
 * the coarse-level executor's tails, the neighbouring launches). The
 * solve's result does not depend on the shapes; h's blocks end as after
 * mg_fmg. Set the right-hand sides first. Synchronizes `stream`. out
 * (nullable): the chosen shapes, the solve time with each level's pick in
 * its last comparison (star_us, transfer_us) and with the default shape in
 * its first (*_default_us).                                               */
int mg_autotune_solve(mg_hierarchy* h, int reps, void* stream, mg_tune_report* out);

/* Launch-shape tuning (process-wide; results do not depend on it):
 * "star2d_rows" / "star3d_rows" = rows or planes one wave of the star
 * stencil kernels marches on large grids, "star2d_small_n" /
 * "star3d_small_n" = grid size below which every wave takes a single row
 * (values >= 1; "star2d_rows" = 0 restores the default, rows = n^2 / 2^18
 * rounded down to a power of two in [1, 64]); "transfer_rows" = coarse
 * rows (2D) or planes (3D) one wave of the restriction / prolongation
 * kernels marches (0, the default: a power of two in [1, 32] that gives a
 * few thousand waves); "level_rows_clear" (any value) forgets the per-level
 * shapes mg_autotune chose; "exec_max_points" = largest grid (in interior points) whose
 * level runs inside the one-workgroup coarse-level programs a hierarchy
 * records at creation (0 = never; read by mg_hierarchy_bytes/create);
 * "tiles2d_rows" = rows one wave of the 2D tiled stencil marches (tiles of
 * at least 4 points; even values 2..1024, 0 = chosen from the grid size);
 * "diagnostics" = 1: hierarchies created while it is set keep the solve
 * diagnostics of mg_diag_read (0, the default: none, and no cost; read by
 * mg_hierarchy_bytes/create, which must see the same value);
 * "stream_copy_blocks" / "stream_copy_per_thread": the shape of
 * bfp_stream_copy (values >= 1);
 * "fuse_relax_res" = 1: a 2D V-cycle's relaxation from zero and the
 * residual after it (both nnqcomp, 32-bit storage, no diagnostics) run as
 * one launch on the launched levels whose grids have at most
 * "relax_res_max_n" points a side (default 255); 0 (the default): two
 * launches (the same results; measured faster on MI355X, the fused kernel
 * doing twice the arithmetic per point); "relax_res_rows" = rows one wave
 * of that launch marches (0, the default: from the grid size);
 * "fe_one_launch" = the largest output (points, at most 4096, the
 * default) of a finite-element op that runs both qcomp passes in one
 * single-workgroup launch (0: always two launches; the same results);
 * "fe_program" = 1 (the default): fe_fmg runs the whole solve as the one
 * single-workgroup program fe_hierarchy_create recorded (hierarchies whose
 * every block has at most 4096 unknowns); 0: op by op (the same results). */
int bfp_tuning_set(const char* key, int value);

/* Current value of a tuning key (the keys of bfp_tuning_set) into *value.
 * BFP_EINVAL for an unknown key or a NULL argument.                      */
int bfp_tuning_get(const char* key, int* value);

/* Human-readable description of the last error on this thread.           */
const char* bfp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BFPMG_H */
