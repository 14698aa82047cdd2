// C-ABI entry points of the BFP library: argument validation, the integer
// budget checks that keep every exact intermediate inside 62 bits, and the
// dispatch of each operation onto its kernels.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"
#include "kernels.hpp"

namespace bfpk {

static thread_local std::string g_last_error;

// Launch-shape tuning of the star kernels: rows (2D) or planes (3D) one
// wave marches. Measured on MI355X: a march pays about one memory latency
// per 4-line batch, so longer marches win only while the grid still offers
// ~1-2 waves per SIMD. The default picks rows = n^2 / 2^18 (2D), clamped to
// [1, 64] and rounded down to a power of two; the tuning keys override it.
static int g_star2d_rows_large = 0, g_star2d_small_n = 0;
static int g_star3d_rows_large = 32, g_star3d_small_n = 64;

// Coarse-level executor: programs are recorded for the levels whose grids
// hold at most this many points (0 disables the executor).
static int g_exec_max_points = 4096;
static int g_fuse_relax_res = 0;
static int g_relax_res_rows = 0;
static int g_relax_res_max_n = 255;
static int g_stream_copy_blocks = 1024;
static int g_stream_copy_per_thread = 4;
static int g_fe_one_launch = 4096;
int fe_one_launch() { return g_fe_one_launch; }
static int g_fe_program = 1;
bool fe_program() { return g_fe_program != 0; }
bool fuse_relax_res() { return g_fuse_relax_res != 0; }
int relax_res_rows() { return g_relax_res_rows; }
int relax_res_max_n() { return g_relax_res_max_n; }

int exec_max_points() { return g_exec_max_points; }

// Rows one wave of the 2D tiled stencil kernel (tiles of >= 4 points)
// marches (0: chosen from the grid size).
static int g_tiles_rows = 0;

int tiles_rows() { return g_tiles_rows; }

// Hierarchies created while this is set keep solve diagnostics.
static int g_diagnostics = 0;

bool diagnostics_on() { return g_diagnostics != 0; }

// While a sink is installed (on this host thread), the operations append
// their launch descriptions to it instead of launching.
static thread_local std::vector<ExecOp>* g_rec = nullptr;

void record_into(std::vector<ExecOp>* sink) { g_rec = sink; }
bool recording() { return g_rec != nullptr; }

// While set (on this host thread), the operations count their diagnostics
// into these kDiagBins counters (and carry their estimate in qcomp mode).
static thread_local int64_t* g_diag = nullptr;

void set_diag_row(int64_t* row) { g_diag = row; }

// While set (on this host thread), the operations reduce their outputs
// through these per-block slots (2 * kMaxSlotBlocks int64).
static thread_local int64_t* g_slots = nullptr;

void set_slots(int64_t* slots) { g_slots = slots; }

static int64_t out_n(const StarLaunch& l) { return l.n; }
static int64_t out_n(const TransferLaunch& l) { return l.n_out; }
static int64_t out_n(const PointLaunch& l) { return l.n; }
static void put_launch(ExecOp& e, const StarLaunch& l) { e.kind = kExStar; e.u.star = l; }
static void put_launch(ExecOp& e, const TransferLaunch& l) { e.kind = kExTransfer; e.u.tr = l; }
static void put_launch(ExecOp& e, const PointLaunch& l) { e.kind = kExPoint; e.u.pt = l; }

template <typename L>
static int record(const L& launch, int exec_mode) {
  if (out_n(launch) >= kExecMaxN)
    return fail(BFP_ESHAPE, "grid too large for the coarse-level executor");
  ExecOp e;
  std::memset(&e, 0, sizeof e);
  put_launch(e, launch);
  e.mode = exec_mode;
  g_rec->push_back(e);
  return BFP_OK;
}

int exec_assign_slots(std::vector<ExecOp>& ops, std::vector<int64_t*>& metas) {
  metas.clear();
  auto slot_of = [&](const int64_t* p) -> int16_t {
    if (!p) return -1;
    for (size_t i = 0; i < metas.size(); ++i)
      if (metas[i] == p) return (int16_t)i;
    metas.push_back(const_cast<int64_t*>(p));
    return (int16_t)(metas.size() - 1);
  };
  for (ExecOp& e : ops) {
    const OpArgs* a = e.kind == kExStar       ? &e.u.star.op
                      : e.kind == kExTransfer ? &e.u.tr.op
                      : e.kind == kExPoint    ? &e.u.pt.op
                                              : nullptr;
    for (int i = 0; i < 5; ++i) e.slot[i] = -1;
    if (a) {
      e.slot[0] = slot_of(a->x_meta);
      e.slot[1] = a->has_y ? slot_of(a->y_meta) : -1;
      e.slot[2] = slot_of(a->z_meta);
      e.slot[3] = slot_of(a->g.a);
      e.slot[4] = slot_of(a->g.b);
    } else if (e.kind == kExConv) {
      e.slot[2] = slot_of(e.u.conv.meta);
    } else {
      e.slot[2] = slot_of(e.u.zero.meta);
    }
    if (metas.size() > (size_t)kExecMaxMeta)
      return fail(BFP_EINVAL, "a recorded program touches more than %d blocks", kExecMaxMeta);
  }
  return BFP_OK;
}

// Grid transfers: coarse rows (2D) / planes (3D) one wave marches; the
// default aims at a few thousand waves per launch (0 = default).
static int g_transfer_rows = 0;

// Per-level shapes chosen by mg_autotune, [ndim - 2][level j] for grids of
// n = 2^j - 1 points per dimension (transfers: the fine grid's level); 0 =
// the default. An explicit tuning key takes precedence.
static int g_level_rows[2][2][MG_MAX_LEVELS + 1];   // [kind: star, transfer]

static int pow2_level(int64_t n) {
  for (int j = 1; j <= MG_MAX_LEVELS; ++j)
    if (n == ((int64_t)1 << j) - 1) return j;
  return 0;
}

void set_level_rows(int kind, int ndim, int level, int rows) {
  if ((kind == 0 || kind == 1) && (ndim == 2 || ndim == 3) && level >= 1 && level <= MG_MAX_LEVELS)
    g_level_rows[kind][ndim - 2][level] = rows;
}

int level_rows(int kind, int ndim, int level) {
  if ((kind == 0 || kind == 1) && (ndim == 2 || ndim == 3) && level >= 1 && level <= MG_MAX_LEVELS)
    return g_level_rows[kind][ndim - 2][level];
  return 0;
}

static int transfer_rows(int ndim, int64_t n_out, int64_t nc) {
  if (g_transfer_rows > 0) return g_transfer_rows;
  const int tuned = level_rows(1, ndim, pow2_level(2 * nc + 1));
  if (tuned > 0) return tuned;
  const int64_t segs = (n_out + 2 + 255) / 256;
  const int64_t lines = ndim == 2 ? segs * (nc + 1) : segs * (nc + 1) * (nc + 1);
  int rows = 1;
  while (rows < 32 && (int64_t)rows * 2 * 4096 <= lines) rows *= 2;
  return rows;
}

static int star_rows(int ndim, int64_t n) {
  const int tuned = level_rows(0, ndim, pow2_level(n));
  if (ndim == 2) {
    if (g_star2d_rows_large > 0) return n < g_star2d_small_n ? 1 : g_star2d_rows_large;
    if (tuned > 0) return tuned;
    int64_t r = n * n / (1 << 18);
    int rows = 1;
    while (rows * 2 <= r && rows < 64) rows *= 2;
    return rows;
  }
  if (tuned > 0 && g_star3d_rows_large == 32 && g_star3d_small_n == 64) return tuned;
  return n < g_star3d_small_n ? 1 : g_star3d_rows_large;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return BFP_OK;
  return fail(BFP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// rows start on 128-byte boundaries (a block is 256-byte aligned), so a
// wave's 1 KB column segment covers whole cache lines
int64_t pitch_for(int64_t n, int bits) {
  const int64_t per128 = 1024 / bits;  // elements per 128 bytes
  return ((n + 2 + per128 - 1) / per128) * per128;
}

int64_t rows_for(int ndim, int64_t n) { return ndim == 3 ? (n + 2) * (n + 2) : (n + 2); }

int check_vec(const bfp_vec* v, const char* name) {
  if (!v) return fail(BFP_EINVAL, "%s is NULL", name);
  if (!v->mant || !v->meta) return fail(BFP_EINVAL, "%s has a NULL pointer", name);
  if (v->storage_bits != 8 && v->storage_bits != 16 && v->storage_bits != 32)
    return fail(BFP_EWIDTH, "%s: storage_bits must be 8, 16 or 32", name);
  if (v->w < 1 || v->w > v->storage_bits)
    return fail(BFP_EWIDTH, "%s: width %d outside 1..%d", name, v->w, v->storage_bits);
  if (v->ndim != 2 && v->ndim != 3) return fail(BFP_ESHAPE, "%s: ndim must be 2 or 3", name);
  if (v->n < 1) return fail(BFP_ESHAPE, "%s: n must be >= 1", name);
  const int64_t per16 = 128 / v->storage_bits;
  if (v->pitch < v->n + 2 || v->pitch % per16)
    return fail(BFP_ESHAPE, "%s: pitch %lld is not a multiple of %lld that holds n+2", name,
                (long long)v->pitch, (long long)per16);
  if ((uintptr_t)v->mant % 16) return fail(BFP_EINVAL, "%s: mantissas not 16-byte aligned", name);
  if ((uintptr_t)v->meta % 8) return fail(BFP_EINVAL, "%s: meta not 8-byte aligned", name);
  return BFP_OK;
}

static int check_scalar(const bfp_scalar* s, const char* name, int max_bits) {
  if (!s) return fail(BFP_EINVAL, "%s is NULL", name);
  const int64_t lim = (int64_t)1 << (max_bits - 1);
  if (s->m < -lim || s->m >= lim)
    return fail(BFP_EWIDTH, "%s: mantissa outside %d bits", name, max_bits);
  if (s->exp < -(1ll << 40) || s->exp > (1ll << 40))
    return fail(BFP_EINVAL, "%s: exponent out of range", name);
  return BFP_OK;
}

int fill_gamma(const bfp_gamma* g, int mode, GammaArgs* out) {
  std::memset(out, 0, sizeof *out);
  // qcomp needs no estimate; with diagnostics on it carries the one given,
  // for the window-gap count
  if (mode != BFP_SATURATE && !(g && g_diag)) return BFP_OK;
  if (!g) return fail(BFP_EINVAL, "BFP_SATURATE needs a gamma estimate");
  out->rule = g->rule;
  out->a = g->a_meta;
  out->b = g->b_meta;
  out->cm = g->c.m;
  out->ce = g->c.exp;
  switch (g->rule) {
    case BFP_GAMMA_NORM:
      if (!g->a_meta) return fail(BFP_EINVAL, "gamma NORM needs a_meta");
      if (g->c.m <= 0 || g->c.m >= (1ll << 24)) return fail(BFP_EINVAL, "gamma NORM needs 0 < c.m < 2^24");
      break;
    case BFP_GAMMA_SUM:
      if (!g->a_meta || !g->b_meta) return fail(BFP_EINVAL, "gamma SUM needs a_meta and b_meta");
      break;
    case BFP_GAMMA_EXPLICIT:
      if (g->c.m < 0) return fail(BFP_EINVAL, "gamma EXPLICIT needs c >= 0");
      break;
    default:
      return fail(BFP_EINVAL, "unknown gamma rule %d", g->rule);
  }
  if (g->c.exp < -(1ll << 40) || g->c.exp > (1ll << 40))
    return fail(BFP_EINVAL, "gamma exponent out of range");
  return BFP_OK;
}

static bool is_star(const bfp_stencil* A) {
  for (int i = 0; i < (A->ndim == 3 ? 27 : 9); ++i) {
    int o[3];
    if (A->ndim == 3) { o[0] = i / 9 - 1; o[1] = (i / 3) % 3 - 1; o[2] = i % 3 - 1; }
    else { o[0] = 0; o[1] = i / 3 - 1; o[2] = i % 3 - 1; }
    const int l1 = std::abs(o[0]) + std::abs(o[1]) + std::abs(o[2]);
    if (l1 > 1 && A->taps[i] != 0) return false;
  }
  return true;
}

static int tap(const bfp_stencil* A, int oz, int oy, int ox) {
  return A->ndim == 3 ? A->taps[((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1)]
                      : A->taps[(oy + 1) * 3 + (ox + 1)];
}

// bit bound k of a term: |m| * tsum * 2^(w-1) < 2^k bounds |m * sum t x| over
// w-bit mantissas x (tsum = sum of |taps|, 1 for a pointwise term)
static int term_bits(int64_t m, uint64_t tsum, int w) {
  unsigned __int128 b = (unsigned __int128)(m < 0 ? -(unsigned __int128)m : (unsigned __int128)m) *
                        tsum << (w - 1);
  int k = 0;
  while (b >> k) ++k;
  return k;
}

static uint64_t tap_sum(const int32_t* t, int count) {
  uint64_t s = 0;
  for (int i = 0; i < count; ++i) s += (uint64_t)(t[i] < 0 ? -(int64_t)t[i] : t[i]);
  return s;
}

// |alpha| * sum |t| * 2^(w-1) < 2^61 and |beta| 2^(wy-1) < 2^61
static int check_budget(const bfp_stencil* A, const bfp_vec* x, int64_t alpha_m,
                        const bfp_vec* y, int64_t beta_m, bool* wide) {
  long double gb = 0;
  if (A) {
    for (int i = 0; i < (A->ndim == 3 ? 27 : 9); ++i) gb += std::abs((long double)A->taps[i]);
  } else {
    gb = 1;
  }
  gb *= ldexpl(1.0L, x->w - 1);
  if (wide) *wide = !(gb < ldexpl(1.0L, 31));
  if (std::abs((long double)alpha_m) * gb >= ldexpl(1.0L, 61))
    return fail(BFP_EWIDTH, "alpha * A x may exceed the 61-bit exact budget");
  if (y && std::abs((long double)beta_m) * ldexpl(1.0L, y->w - 1) >= ldexpl(1.0L, 61))
    return fail(BFP_EWIDTH, "beta * y may exceed the 61-bit exact budget");
  return BFP_OK;
}

static void fill_common(OpArgs* op, int w_out, const bfp_vec* x, const bfp_vec* y,
                        const bfp_vec* z) {
  op->w_out = w_out;
  op->x_meta = x->meta;
  op->y_meta = y ? y->meta : x->meta;
  op->z_meta = z->meta;
  op->has_y = y != nullptr;
  op->lo = -((int64_t)1 << (w_out - 1));
  op->hi = ((int64_t)1 << (w_out - 1)) - 1;
  op->diag = g_diag;
  op->slots = g_slots;
}

// While set, a star op in saturate mode is prepared into *g_take_star
// instead of launched (star_prepare_sat).
static thread_local StarLaunch* g_take_star = nullptr;

// Run one op in the requested mode: nnqcomp in one launch, qcomp as the
// mu* pass followed by the output pass.
template <typename L, typename F>
static int run_modes(L& launch, int mode, hipStream_t s, F&& go) {
  if (g_rec) return record(launch, mode == BFP_SATURATE ? kModeSat : kExModeQ);
  if constexpr (std::is_same<L, StarLaunch>::value) {
    if (g_take_star) {
      if (mode != BFP_SATURATE) return fail(BFP_EINVAL, "only saturate-mode ops are prepared");
      launch.op.mode = kModeSat;
      *g_take_star = launch;
      return BFP_OK;
    }
  }
  int rc;
  if (mode == BFP_SATURATE) {
    launch.op.mode = kModeSat;
    if ((rc = hip_check(go(launch), "kernel launch"))) return rc;
    if (launch.op.diag)
      rc = hip_check(launch_diag_sat(launch.op.diag, launch.op.z_meta, s), "diagnostics");
    return rc;
  }
  launch.op.mode = kModeQ1;
  if ((rc = hip_check(go(launch), "kernel launch (qcomp pass 1)"))) return rc;
  if (launch.op.diag && (rc = hip_check(launch_diag_q(launch.op, s), "diagnostics"))) return rc;
  launch.op.mode = kModeQ2;
  return hip_check(go(launch), "kernel launch (qcomp pass 2)");
}

int stencil_apply_impl(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                       const bfp_scalar* beta, const bfp_vec* y, int w_out, int mode,
                       const bfp_gamma* gamma, bfp_vec* z, hipStream_t s, int rows) {
  int rc;
  if (!A) return fail(BFP_EINVAL, "stencil is NULL");
  if ((rc = check_vec(x, "x")) || (rc = check_vec(z, "z"))) return rc;
  if (y && (rc = check_vec(y, "y"))) return rc;
  if (mode != BFP_NORMALIZE && mode != BFP_SATURATE) return fail(BFP_EINVAL, "bad mode %d", mode);
  if (w_out < 1 || w_out > z->w)
    return fail(BFP_EWIDTH, "w_out %d outside 1..%d (the width of z)", w_out, z->w);
  if (A->ndim != x->ndim || x->ndim != z->ndim || (y && y->ndim != z->ndim))
    return fail(BFP_ESHAPE, "dimension mismatch");
  if (y && y->n != z->n) return fail(BFP_ESHAPE, "y and z differ in size");
  if (x->mant == z->mant || x->meta == z->meta)
    return fail(BFP_EINVAL, "the output of a stencil may not alias its input");
  for (int i = 0; i < 27; ++i)
    if (A->taps[i] < -(1 << 23) || A->taps[i] >= (1 << 23))
      return fail(BFP_EWIDTH, "stencil taps must fit 24 bits");
  if (A->exp < -(1ll << 40) || A->exp > (1ll << 40)) return fail(BFP_EINVAL, "stencil exponent out of range");
  bfp_scalar one{1, 0, 2};
  const bfp_scalar* al = alpha ? alpha : &one;
  const bfp_scalar* be = beta ? beta : &one;
  if ((rc = check_scalar(al, "alpha", 32))) return rc;
  if (y && (rc = check_scalar(be, "beta", 32))) return rc;
  bool wide = true;
  if ((rc = check_budget(A, x, al->m, y, be->m, &wide))) return rc;

  // alpha * (A x) = (alpha_m A) x: fold alpha's mantissa into the taps when
  // every product fits the 24-bit tap range, so the kernels skip a 64-bit
  // multiply per point (the exact value is unchanged)
  int32_t taps[27];
  int64_t am = al->m;
  bool fold = true;
  for (int i = 0; i < 27; ++i) {
    const int64_t t = (int64_t)A->taps[i] * al->m;
    if (t < -(1 << 23) || t >= (1 << 23)) fold = false;
  }
  for (int i = 0; i < 27; ++i) taps[i] = fold ? (int32_t)(A->taps[i] * al->m) : A->taps[i];
  if (fold) am = 1;
  bfp_stencil Af = *A;
  for (int i = 0; i < 27; ++i) Af.taps[i] = taps[i];
  A = &Af;
  {
    // int32 accumulation of the (folded) stencil sum only when it cannot overflow
    long double gb = 0;
    for (int i = 0; i < 27; ++i) gb += std::abs((long double)taps[i]);
    wide = !(gb * ldexpl(1.0L, x->w - 1) < ldexpl(1.0L, 31));
  }

  OpArgs op{};
  fill_common(&op, w_out, x, y, z);
  op.e_A = A->exp;
  op.alpha_m = am;
  op.alpha_e = al->exp;
  op.beta_m = y ? be->m : 0;
  op.beta_e = y ? be->exp : 0;
  op.abits = term_bits(am, tap_sum(taps, 27), x->w);
  op.bbits = y ? term_bits(be->m, 1, y->w) : 0;
  if ((rc = fill_gamma(gamma, mode, &op.g))) return rc;

  if (A->kind == BFP_STENCIL_A) {
    if (x->n != z->n) return fail(BFP_ESHAPE, "A: x and z differ in size");
    if (!is_star(A))
      return fail(BFP_EINVAL, "same-grid stencils must be star-shaped (centre and faces)");
    StarLaunch L{};
    L.op = op;
    L.x = x->mant;
    L.y = y ? y->mant : nullptr;
    L.z = z->mant;
    L.ndim = x->ndim;
    L.n = x->n;
    L.px = x->pitch;
    L.py = y ? y->pitch : x->pitch;
    L.pz = z->pitch;
    L.taps[0] = tap(A, 0, 0, 0);
    L.taps[1] = tap(A, 0, 0, -1);
    L.taps[2] = tap(A, 0, 0, 1);
    L.taps[3] = tap(A, 0, -1, 0);
    L.taps[4] = tap(A, 0, 1, 0);
    L.taps[5] = A->ndim == 3 ? tap(A, -1, 0, 0) : 0;
    L.taps[6] = A->ndim == 3 ? tap(A, 1, 0, 0) : 0;
    L.xbits = x->storage_bits;
    L.ybits = y ? y->storage_bits : 32;
    L.zbits = z->storage_bits;
    L.wide = wide;
    L.y_is_x = y && y->mant == x->mant && y->storage_bits == x->storage_bits &&
               y->pitch == x->pitch;
    L.rows = rows > 0 ? rows : star_rows(x->ndim, x->n);
    {
      const int64_t segs = (x->n + 1 + 255) / 256;
      L.wx = segs >= 4 ? 4 : (segs >= 2 ? 2 : 1);
    }
    return run_modes(L, mode, s, [&](StarLaunch& l) { return launch_star(l, s); });
  }
  if (A->kind == BFP_STENCIL_R || A->kind == BFP_STENCIL_P) {
    const bfp_vec* fine = A->kind == BFP_STENCIL_R ? x : z;
    const bfp_vec* coarse = A->kind == BFP_STENCIL_R ? z : x;
    if (fine->n != 2 * coarse->n + 1)
      return fail(BFP_ESHAPE, "transfer: fine n must be 2 * coarse n + 1 (%d vs %d)", fine->n,
                  coarse->n);
    TransferLaunch L{};
    L.op = op;
    L.kind = A->kind;
    L.x = x->mant;
    L.y = y ? y->mant : nullptr;
    L.z = z->mant;
    L.ndim = x->ndim;
    L.n_in = x->n;
    L.n_out = z->n;
    L.px = x->pitch;
    L.py = y ? y->pitch : z->pitch;
    L.pz = z->pitch;
    for (int i = 0; i < 27; ++i) L.taps[i] = A->taps[i];
    L.xbits = x->storage_bits;
    L.ybits = y ? y->storage_bits : 32;
    L.zbits = z->storage_bits;
    L.rows = transfer_rows(x->ndim, z->n, coarse->n);
    return run_modes(L, mode, s, [&](TransferLaunch& l) { return launch_transfer(l, s); });
  }
  return fail(BFP_EINVAL, "unknown stencil kind %d", A->kind);
}

int star_prepare_sat(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                     const bfp_scalar* beta, const bfp_vec* y, int w_out,
                     const bfp_gamma* gamma, bfp_vec* z, StarLaunch* out) {
  if (A && A->kind != BFP_STENCIL_A) return fail(BFP_EINVAL, "not a same-grid stencil");
  StarLaunch L{};
  g_take_star = &L;
  const int rc = stencil_apply_impl(A, x, alpha, beta, y, w_out, BFP_SATURATE, gamma, z, nullptr, 0);
  g_take_star = nullptr;
  if (!rc) *out = L;
  return rc;
}

int point_impl(const bfp_scalar* alpha, const bfp_vec* x, const bfp_scalar* beta,
               const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma, bfp_vec* z,
               hipStream_t s, int forced_mode) {
  int rc;
  if ((rc = check_vec(x, "x")) || (rc = check_vec(z, "z"))) return rc;
  if (y && (rc = check_vec(y, "y"))) return rc;
  if (w_out < 1 || w_out > z->w)
    return fail(BFP_EWIDTH, "w_out %d outside 1..%d (the width of z)", w_out, z->w);
  if (x->ndim != z->ndim || x->n != z->n || (y && (y->ndim != z->ndim || y->n != z->n)))
    return fail(BFP_ESHAPE, "pointwise operands differ in shape");
  if ((rc = check_scalar(alpha, "alpha", 32))) return rc;
  if (y && (rc = check_scalar(beta, "beta", 32))) return rc;
  if ((rc = check_budget(nullptr, x, alpha->m, y, y ? beta->m : 0, nullptr))) return rc;
  PointLaunch L{};
  fill_common(&L.op, w_out, x, y, z);
  L.op.alpha_m = alpha->m;
  L.op.alpha_e = alpha->exp;
  L.op.beta_m = y ? beta->m : 0;
  L.op.beta_e = y ? beta->exp : 0;
  L.op.abits = term_bits(alpha->m, 1, x->w);
  L.op.bbits = y ? term_bits(beta->m, 1, y->w) : 0;
  L.x = x->mant;
  L.y = y ? y->mant : nullptr;
  L.z = z->mant;
  L.ndim = x->ndim;
  L.n = x->n;
  L.px = x->pitch;
  L.py = y ? y->pitch : x->pitch;
  L.pz = z->pitch;
  L.xbits = x->storage_bits;
  L.ybits = y ? y->storage_bits : 32;
  L.zbits = z->storage_bits;
  if (forced_mode == kModeNormMeta || forced_mode == kModeAssign) {
    L.op.mode = forced_mode;
    if (g_rec) return record(L, forced_mode);
    return hip_check(launch_point(L, s), "pointwise launch");
  }
  if (mode != BFP_NORMALIZE && mode != BFP_SATURATE) return fail(BFP_EINVAL, "bad mode %d", mode);
  if ((rc = fill_gamma(gamma, mode, &L.op.g))) return rc;
  return run_modes(L, mode, s, [&](PointLaunch& l) { return launch_point(l, s); });
}

}  // namespace bfpk

namespace bfpk {

int from_f64_impl(const double* src_dev, const double* const* table_dev, int index,
                  int64_t log2_scale, bfp_vec* dst, hipStream_t s) {
  int rc = check_vec(dst, "dst");
  if (rc) return rc;
  if (!src_dev && !table_dev) return fail(BFP_EINVAL, "src is NULL");
  if (log2_scale < -(1ll << 30) || log2_scale > (1ll << 30)) return fail(BFP_EINVAL, "log2_scale out of range");
  ConvertLaunch L{};
  L.src = src_dev;
  L.src_table = table_dev;
  L.table_index = index;
  L.mant = dst->mant;
  L.meta = dst->meta;
  L.ndim = dst->ndim;
  L.n = dst->n;
  L.pitch = dst->pitch;
  L.bits = dst->storage_bits;
  L.w = dst->w;
  L.log2_scale = log2_scale;
  return hip_check(launch_from_f64(L, s), "bfp_vec_from_f64");
}

int to_f64_impl(const bfp_vec* src, double* dst_dev, double* const* table_dev, int index,
                hipStream_t s) {
  int rc = check_vec(src, "src");
  if (rc) return rc;
  if (!dst_dev && !table_dev) return fail(BFP_EINVAL, "dst is NULL");
  ConvertLaunch L{};
  L.dst = dst_dev;
  L.dst_table = table_dev;
  L.table_index = index;
  L.mant = src->mant;
  L.meta = src->meta;
  L.ndim = src->ndim;
  L.n = src->n;
  L.pitch = src->pitch;
  L.bits = src->storage_bits;
  L.w = src->w;
  return hip_check(launch_to_f64(L, s), "bfp_vec_to_f64");
}

}  // namespace bfpk

using namespace bfpk;

extern "C" {

const char* bfp_last_error(void) { return g_last_error.c_str(); }

int bfp_layout(int ndim, int n, int storage_bits, int64_t* pitch, size_t* bytes) {
  if (ndim != 2 && ndim != 3) return fail(BFP_ESHAPE, "ndim must be 2 or 3");
  if (n < 1) return fail(BFP_ESHAPE, "n must be >= 1");
  if (storage_bits != 8 && storage_bits != 16 && storage_bits != 32)
    return fail(BFP_EWIDTH, "storage_bits must be 8, 16 or 32");
  const int64_t p = pitch_for(n, storage_bits);
  if (pitch) *pitch = p;
  if (bytes) *bytes = (size_t)(p * rows_for(ndim, n) * (storage_bits / 8));
  return BFP_OK;
}

int bfp_vec_init(const bfp_vec* v, void* stream) {
  int rc = check_vec(v, "v");
  if (rc) return rc;
  const size_t bytes = (size_t)(v->pitch * rows_for(v->ndim, v->n) * (v->storage_bits / 8));
  if (g_rec) {
    ExecOp e;
    std::memset(&e, 0, sizeof e);
    e.kind = kExZero;
    e.u.zero = ZeroOp{v->mant, v->meta, (int64_t)bytes, (int64_t)(1 - v->w)};
    g_rec->push_back(e);
    return BFP_OK;
  }
  return hip_check(launch_init(v->mant, bytes, v->meta, 1 - v->w, (hipStream_t)stream),
                   "bfp_vec_init");
}

int bfp_meta_reset(int64_t* meta_dev, void* stream) {
  if (!meta_dev) return fail(BFP_EINVAL, "meta is NULL");
  return hip_check(launch_meta_reset(meta_dev, (hipStream_t)stream), "bfp_meta_reset");
}

int bfp_vec_from_f64(const double* src_dev, int64_t log2_scale, bfp_vec* dst, void* stream) {
  if (!src_dev) return fail(BFP_EINVAL, "src is NULL");
  return from_f64_impl(src_dev, nullptr, 0, log2_scale, dst, (hipStream_t)stream);
}

int bfp_vec_to_f64(const bfp_vec* src, double* dst_dev, void* stream) {
  if (!dst_dev) return fail(BFP_EINVAL, "dst is NULL");
  return to_f64_impl(src, dst_dev, nullptr, 0, (hipStream_t)stream);
}

int bfp_vec_check(const bfp_vec* v, void* stream) {
  int rc = check_vec(v, "v");
  if (rc) return rc;
  int64_t flags = 0;
  rc = hip_check(hipMemcpyAsync(&flags, v->meta + BFP_META_FLAGS, sizeof flags,
                                hipMemcpyDeviceToHost, (hipStream_t)stream),
                 "bfp_vec_check copy");
  if (rc) return rc;
  if ((rc = hip_check(hipStreamSynchronize((hipStream_t)stream), "bfp_vec_check sync"))) return rc;
  if (flags & 1) return fail(BFP_ENONFINITE, "non-finite FP64 input");
  return BFP_OK;
}

int bfp_stencil_apply(const bfp_stencil* A, const bfp_vec* x, const bfp_scalar* alpha,
                      const bfp_scalar* beta, const bfp_vec* y, int w_out, int mode,
                      const bfp_gamma* gamma, bfp_vec* z, void* stream) {
  return stencil_apply_impl(A, x, alpha, beta, y, w_out, mode, gamma, z, (hipStream_t)stream, 0);
}

int bfp_residual(const bfp_stencil* A, const bfp_vec* x, const bfp_vec* b, int w_out, int mode,
                 const bfp_gamma* gamma, bfp_vec* r, void* stream) {
  if (!b) return fail(BFP_EINVAL, "b is NULL");
  bfp_scalar one{1, 0, 2}, mone{-1, 0, 1};
  return stencil_apply_impl(A, x, &one, &mone, b, w_out, mode, gamma, r, (hipStream_t)stream, 0);
}

int bfp_axpy(const bfp_scalar* alpha, const bfp_vec* x, const bfp_scalar* beta, const bfp_vec* y,
             int w_out, int mode, const bfp_gamma* gamma, bfp_vec* z, void* stream) {
  if (!y) return fail(BFP_EINVAL, "y is NULL");
  return point_impl(alpha, x, beta, y, w_out, mode, gamma, z, (hipStream_t)stream, -1);
}

int bfp_sub(const bfp_vec* x, const bfp_vec* y, int w_out, int mode, const bfp_gamma* gamma,
            bfp_vec* z, void* stream) {
  if (!y) return fail(BFP_EINVAL, "y is NULL");
  bfp_scalar one{1, 0, 2}, mone{-1, 0, 1};
  return point_impl(&one, x, &mone, y, w_out, mode, gamma, z, (hipStream_t)stream, -1);
}

int bfp_normalize(const bfp_vec* in, int w_out, bfp_vec* out, void* stream) {
  bfp_scalar one{1, 0, 2};
  return point_impl(&one, in, nullptr, nullptr, w_out, BFP_NORMALIZE, nullptr, out,
                    (hipStream_t)stream, kModeNormMeta);
}

int bfp_saturate_truncate(const bfp_vec* in, int w_out, const bfp_gamma* gamma, bfp_vec* out,
                          void* stream) {
  bfp_scalar one{1, 0, 2};
  return point_impl(&one, in, nullptr, nullptr, w_out, BFP_SATURATE, gamma, out,
                    (hipStream_t)stream, -1);
}

int bfp_tuning_set(const char* key, int value) {
  if (!key) return fail(BFP_EINVAL, "key is NULL");
  if (value < 0 || value > 1 << 20) return fail(BFP_EINVAL, "value out of range");
  const std::string k(key);
  if (k == "exec_max_points") { g_exec_max_points = value; return BFP_OK; }
  if (k == "diagnostics") {
    if (value > 1) return fail(BFP_EINVAL, "diagnostics is 0 or 1");
    g_diagnostics = value;
    return BFP_OK;
  }
  // 2D: rows 0 restores the size heuristic (then small_n is not read)
  if (k == "star2d_rows") { g_star2d_rows_large = value; return BFP_OK; }
  if (k == "transfer_rows") { g_transfer_rows = value; return BFP_OK; }
  if (k == "level_rows_clear") {   // forget the shapes mg_autotune chose
    std::memset(g_level_rows, 0, sizeof g_level_rows);
    return BFP_OK;
  }
  if (k == "star2d_small_n") { g_star2d_small_n = value; return BFP_OK; }
  if (k == "fuse_relax_res") {
    if (value > 1) return fail(BFP_EINVAL, "fuse_relax_res is 0 or 1");
    g_fuse_relax_res = value;
    return BFP_OK;
  }
  if (k == "relax_res_max_n") { g_relax_res_max_n = value; return BFP_OK; }
  if (k == "fe_program") {
    if (value > 1) return fail(BFP_EINVAL, "fe_program is 0 or 1");
    g_fe_program = value;
    return BFP_OK;
  }
  if (k == "fe_one_launch") {
    if (value > 4096) return fail(BFP_EINVAL, "fe_one_launch is at most 4096");
    g_fe_one_launch = value;
    return BFP_OK;
  }
  if (k == "stream_copy_blocks" || k == "stream_copy_per_thread") {
    if (value < 1) return fail(BFP_EINVAL, "value out of range");
    (k == "stream_copy_blocks" ? g_stream_copy_blocks : g_stream_copy_per_thread) = value;
    return BFP_OK;
  }
  if (k == "relax_res_rows") {
    if (value > 1024) return fail(BFP_EINVAL, "relax_res_rows is at most 1024");
    g_relax_res_rows = value;
    return BFP_OK;
  }
  if (k == "tiles2d_rows") {
    if (value > 1024) return fail(BFP_EINVAL, "tiles2d_rows is at most 1024");
    g_tiles_rows = value;
    return BFP_OK;
  }
  if (value < 1) return fail(BFP_EINVAL, "value out of range");
  if (k == "star3d_rows") g_star3d_rows_large = value;
  else if (k == "star3d_small_n") g_star3d_small_n = value;
  else return fail(BFP_EINVAL, "unknown tuning key %s", key);
  return BFP_OK;
}

int bfp_tuning_get(const char* key, int* value) {
  if (!key || !value) return fail(BFP_EINVAL, "NULL argument");
  const std::string k(key);
  if (k == "exec_max_points") *value = g_exec_max_points;
  else if (k == "diagnostics") *value = g_diagnostics;
  else if (k == "star2d_rows") *value = g_star2d_rows_large;
  else if (k == "transfer_rows") *value = g_transfer_rows;
  else if (k == "star2d_small_n") *value = g_star2d_small_n;
  else if (k == "star3d_rows") *value = g_star3d_rows_large;
  else if (k == "star3d_small_n") *value = g_star3d_small_n;
  else if (k == "tiles2d_rows") *value = g_tiles_rows;
  else if (k == "fuse_relax_res") *value = g_fuse_relax_res;
  else if (k == "relax_res_rows") *value = g_relax_res_rows;
  else if (k == "relax_res_max_n") *value = g_relax_res_max_n;
  else if (k == "fe_one_launch") *value = g_fe_one_launch;
  else if (k == "fe_program") *value = g_fe_program;
  else if (k == "stream_copy_blocks") *value = g_stream_copy_blocks;
  else if (k == "stream_copy_per_thread") *value = g_stream_copy_per_thread;
  else return fail(BFP_EINVAL, "unknown tuning key %s", key);
  return BFP_OK;
}

int bfp_vec_assign(bfp_vec* v, int64_t exp, void* stream) {
  int rc = check_vec(v, "v");
  if (rc) return rc;
  if (exp < -(1ll << 40) || exp > (1ll << 40)) return fail(BFP_EINVAL, "exponent out of range");
  PointLaunch L{};
  fill_common(&L.op, v->w, v, nullptr, v);
  L.op.alpha_m = 1;
  L.op.abits = term_bits(1, 1, v->w);
  L.op.assign_exp = exp;
  L.op.mode = kModeAssign;
  L.x = v->mant;
  L.z = v->mant;
  L.ndim = v->ndim;
  L.n = v->n;
  L.px = L.py = L.pz = v->pitch;
  L.xbits = L.zbits = v->storage_bits;
  L.ybits = 32;
  return hip_check(launch_point(L, (hipStream_t)stream), "bfp_vec_assign");
}

int bfp_stream_copy(const void* src_dev, void* dst_dev, int64_t bytes, int nontemporal,
                    void* stream) {
  if (bytes < 0 || bytes % 16) return fail(BFP_EINVAL, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return BFP_OK;
  if (!src_dev || !dst_dev) return fail(BFP_EINVAL, "NULL pointer");
  if (((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15)
    return fail(BFP_EINVAL, "pointers must be 16-byte aligned");
  if (nontemporal != 0 && nontemporal != 1) return fail(BFP_EINVAL, "nontemporal is 0 or 1");
  return hip_check(launch_stream_copy(src_dev, dst_dev, bytes, nontemporal == 1,
                                      g_stream_copy_blocks, g_stream_copy_per_thread,
                                      (hipStream_t)stream),
                   "stream copy");
}

int bfp_dot(const bfp_vec* x, const bfp_vec* y, int64_t* out_dev, void* stream) {
  int rc;
  if ((rc = check_vec(x, "x")) || (rc = check_vec(y, "y"))) return rc;
  if (!out_dev) return fail(BFP_EINVAL, "out is NULL");
  if (x->ndim != y->ndim || x->n != y->n) return fail(BFP_ESHAPE, "dot operands differ in shape");
  DotLaunch L{};
  L.x = x->mant;
  L.y = y->mant;
  L.x_meta = x->meta;
  L.y_meta = y->meta;
  L.out = out_dev;
  L.ndim = x->ndim;
  L.n = x->n;
  L.px = x->pitch;
  L.py = y->pitch;
  L.xbits = x->storage_bits;
  L.ybits = y->storage_bits;
  return hip_check(launch_dot(L, (hipStream_t)stream), "bfp_dot");
}

}  // extern "C"
