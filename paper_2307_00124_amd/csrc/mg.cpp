// BFP multigrid driver: IR, V(nu1, nu2) and FMG (paper Appendix C) built on
// the BFP operations of the library, with the Table 1 estimates evaluated on
// the device from the metadata of earlier results, so a whole solve is one
// stream of kernel launches with no host synchronization.
//
// Operators after the setup S (each level's equations divided by s_j, a
// power of two, so that no BFP division occurs):
//   2D: s_j = 4/h^2      A' = [1; -1/4 x4]        = 2^-2 [4; -1]
//                        R' = P^T                 = 2^-2 [1 2 1; 2 4 2; 1 2 1]
//                        P  = bilinear            = 2^-2 [1 2 1; 2 4 2; 1 2 1]
//   3D: s_j = 8/h^2      A' = [3/4; -1/8 x6]      = 2^-3 [6; -1]
//                        R' = P^T / 2             = 2^-4 * 2^(3 - |o|_1)
//                        P  = trilinear           = 2^-3 * 2^(3 - |o|_1)
// (the 3D scaling is a power of two because diag(A_h) = 6/h^2 would put the
// non-dyadic 1/6 into A'). b'_j = f_j / s_j is an exact exponent shift.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"
#include "kernels.hpp"
#include "vcycle.hpp"

using namespace bfpk;

namespace {

// call sites of the quantizing operations (the rows of the diagnostics)
enum Site { kIrResFirst, kIrRes, kIrCorr, kRelax, kVRes, kRestrict, kVCorr, kFmgProl, kDiagSites };
constexpr size_t kDiagBytes = (size_t)(MG_MAX_LEVELS + 1) * kDiagSites * kDiagBins * sizeof(int64_t);
static_assert(kDiagSites == MG_DIAG_SITES && kDiagBins == MG_DIAG_BINS &&
                  kDiagGapBins == MG_DIAG_GAP_BINS,
              "header diagnostics layout");

struct Level {
  int j;
  int64_t n;
  bfp_vec x, b, r, vr, y, s, t;
};

}  // namespace

namespace {
enum { kPV = 0, kPF = 1, kPI1 = 2, kPI2 = 3, kPIn = 4, kPFc = 5, kPrograms = 6 };
}

// A recorded coarse-level program: ops in the arena, run by one launch of
// the executor; `bytes` is the algorithmic traffic of the ops it stands for.
struct Program {
  ExecOp* ops;
  int count;
  int64_t** metas;   // table of the metadata blocks the ops name by slot
  int nmeta;
  double bytes;
};

struct mg_hierarchy {
  mg_params prm;
  Level lv[MG_MAX_LEVELS + 1];
  bfp_stencil A, R, P;
  bfp_scalar vres;      // (2 c1 + 1) / 4 with the D-scaled c1, exact
  double bytes;
  int64_t launches;
  int Lc;               // levels 1..Lc run inside the programs (0: none)
  // recorded programs: the V-cycle on level Lc from its restricted residual
  // vr, FMG on levels 1..Lc (from x_1 = 0), IR-V iterations on level Lc
  // (the first, the second, any later one), and FMG on levels 1..Lc that
  // first quantizes those levels' right-hand sides from FP64
  Program prog[kPrograms];
  // diagnostic counters [level 0..MG_MAX_LEVELS][site][kDiagBins] in the
  // arena (null for hierarchies that keep none, e.g. the batched ones)
  int64_t* diag = nullptr;
  // per-block partials of the launched operations' output reductions
  // (2 * kMaxSlotBlocks int64; null for batched hierarchies, whose
  // operations all run inside one workgroup)
  int64_t* slots = nullptr;
  // mg_fmg_f64: a second stream (created on first use) that quantizes the
  // finer levels' right-hand sides while the program runs the coarse ones
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  ~mg_hierarchy() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {

// b_j = S_j^-1 f_j: the scaling of level j's FP64 right-hand side, a power
// of two (h_j^2 / 4 in 2D, h_j^2 / 8 in 3D with h_j = 2^-j)
int64_t rhs_shift(int ndim, int j) { return ndim == 2 ? -2 * j - 2 : -2 * j - 3; }

int storage_for(int w, int min_bits) {
  int b = w <= 8 ? 8 : (w <= 16 ? 16 : 32);
  return b < min_bits ? min_bits : b;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------ stencils --

void make_stencils(int ndim, bfp_stencil* A, bfp_stencil* R, bfp_stencil* P) {
  std::memset(A, 0, sizeof *A);
  std::memset(R, 0, sizeof *R);
  std::memset(P, 0, sizeof *P);
  A->ndim = R->ndim = P->ndim = ndim;
  A->kind = BFP_STENCIL_A;
  R->kind = BFP_STENCIL_R;
  P->kind = BFP_STENCIL_P;
  const int nt = ndim == 3 ? 27 : 9;
  for (int i = 0; i < nt; ++i) {
    int l1;
    if (ndim == 3) l1 = std::abs(i / 9 - 1) + std::abs((i / 3) % 3 - 1) + std::abs(i % 3 - 1);
    else l1 = std::abs(i / 3 - 1) + std::abs(i % 3 - 1);
    // interpolation weight 2^-l1 times the common scale
    if (ndim == 2) {
      A->taps[i] = l1 == 0 ? 4 : (l1 == 1 ? -1 : 0);
      R->taps[i] = 4 >> l1;
      P->taps[i] = 4 >> l1;
    } else {
      A->taps[i] = l1 == 0 ? 6 : (l1 == 1 ? -1 : 0);
      R->taps[i] = 8 >> l1;
      P->taps[i] = 8 >> l1;
    }
  }
  if (ndim == 2) {
    A->exp = -2; A->w = 4;
    R->exp = -2; R->w = 4;
    P->exp = -2; P->w = 4;
  } else {
    A->exp = -3; A->w = 4;
    R->exp = -4; R->w = 5;
    P->exp = -3; P->w = 5;
  }
}

// ----------------------------------------------------------- estimates --

bfp_gamma g_norm(const bfp_vec& a, bfp_scalar c) {
  bfp_gamma g{};
  g.rule = BFP_GAMMA_NORM;
  g.a_meta = a.meta;
  g.c = c;
  return g;
}
bfp_gamma g_sum(const bfp_vec& a, const bfp_vec& b) {
  bfp_gamma g{};
  g.rule = BFP_GAMMA_SUM;
  g.a_meta = a.meta;
  g.b_meta = b.meta;
  return g;
}
const bfp_scalar kOne{1, 0, 2};
const bfp_scalar kMinusOne{-1, 0, 1};
const bfp_scalar kFour{1, 2, 2};   // ||R'||_inf = 4 in 2D and 3D

double pts(const bfp_vec& v) {
  double n = (double)v.n;
  return v.ndim == 3 ? n * n * n : n * n;
}
double sz(const bfp_vec& v) { return v.storage_bits / 8.0; }

int mode_for(const mg_hierarchy* h, Site site, bool plain_first2) {
  switch (h->prm.policy) {
    case MG_POLICY_Q: return BFP_NORMALIZE;
    case MG_POLICY_NN: return BFP_SATURATE;
    case MG_POLICY_NN_IR_FIRST_Q:
      return site == kIrResFirst ? BFP_NORMALIZE : BFP_SATURATE;
    case MG_POLICY_NN_IR_FIRST2_Q:
      return (site == kIrResFirst || (site == kIrRes && plain_first2)) ? BFP_NORMALIZE
                                                                        : BFP_SATURATE;
    case MG_POLICY_NN_IR_Q:
      return (site == kIrResFirst || site == kIrRes) ? BFP_NORMALIZE : BFP_SATURATE;
  }
  return BFP_SATURATE;
}

// --------------------------------------------------------------- ops ----

// The diagnostic counters of a call site on the level the call belongs to
// (the recursion level: the input's for a restriction, the output's
// otherwise), while the call is issued; null when the hierarchy keeps none.
int level_of(int64_t n) {
  int j = 0;
  while (((int64_t)1 << j) - 1 < n) ++j;
  return j;
}
// ... and the hierarchy's per-block reduction slots
struct DiagScope {
  DiagScope(mg_hierarchy* h, Site site, int64_t n) {
    set_diag_row(h->diag ? h->diag + ((int64_t)level_of(n) * kDiagSites + site) * kDiagBins
                         : nullptr);
    set_slots(h->slots);
  }
  ~DiagScope() {
    set_diag_row(nullptr);
    set_slots(nullptr);
  }
};

int op_stencil(mg_hierarchy* h, const bfp_stencil* S, const bfp_vec& x, const bfp_scalar* al,
               const bfp_scalar* be, const bfp_vec* y, bfp_vec& z, Site site, int mode,
               const bfp_gamma& g, hipStream_t s) {
  DiagScope diag(h, site, site == kRestrict ? x.n : z.n);
  int rc = stencil_apply_impl(S, &x, al, be, y, z.w, mode, &g, &z, s, 0);
  if (rc) return rc;
  const int passes = mode == BFP_NORMALIZE ? 2 : 1;
  // algorithmic bytes: every input read once (y = x, the relaxation, once;
  // qcomp's second read pass is overhead, not counted), the output written once
  const bool y_own = y && y->mant != x.mant;
  const double rd = pts(x) * sz(x) + (y_own ? pts(*y) * sz(*y) : 0.0);
  h->bytes += rd + pts(z) * sz(z);
  h->launches += passes;
  return BFP_OK;
}

int op_sub(mg_hierarchy* h, const bfp_vec& x, const bfp_vec& y, bfp_vec& z, Site site, int mode,
           const bfp_gamma& g, hipStream_t s) {
  DiagScope diag(h, site, z.n);
  int rc = point_impl(&kOne, &x, &kMinusOne, &y, z.w, mode, &g, &z, s, -1);
  if (rc) return rc;
  const int passes = mode == BFP_NORMALIZE ? 2 : 1;
  h->bytes += pts(x) * sz(x) + pts(y) * sz(y) + pts(z) * sz(z);
  h->launches += passes;
  return BFP_OK;
}

int run_program(mg_hierarchy* h, const Program& pg, hipStream_t s,
                const ExecRhs* rhs = nullptr) {
  int rc = hip_check(launch_exec(pg.ops, pg.count, pg.metas, pg.nmeta, h->prm.ndim, rhs,
                                h->diag != nullptr, s),
                     "coarse-level program");
  if (rc) return rc;
  h->bytes += pg.bytes;
  h->launches += 1;
  return BFP_OK;
}

// The relaxation y = Q(c2 A r + c1 r) and the residual s = Q(A y - r) of
// level l in one launch, when the prepared ops fit the fused kernel
// (*done = false otherwise: nothing was launched).
int relax_res(mg_hierarchy* h, int l, const bfp_vec& rin, hipStream_t s, bool* done) {
  Level& L = h->lv[l];
  const mg_params& p = h->prm;
  *done = false;
  RelaxResLaunch F{};
  const bfp_gamma g1 = g_norm(rin, p.c1), g2 = g_norm(rin, h->vres);
  int rc = star_prepare_sat(&h->A, &rin, &p.c2, &p.c1, &rin, L.y.w, &g1, &L.y, &F.relax);
  if (!rc) rc = star_prepare_sat(&h->A, &L.y, &kOne, &kMinusOne, &rin, L.s.w, &g2, &L.s, &F.res);
  if (rc) return rc;
  // only on grids up to relax_res_max_n a side: on larger grids the two
  // separate kernels run near the bandwidth bound and the fused kernel
  // (twice the arithmetic per point, halo rows computed again) is slower
  // (measured on MI355X: 94 us against 76 us at 4095^2, 36 against 28 at
  // 2047^2); on small grids it saves a launch, but the whole solve still
  // measured 0.3-0.5% slower, so the fusion is off by default
  const int64_t n = L.y.n;
  if (n > relax_res_max_n() || !relax_res_fits(F.relax, F.res)) return BFP_OK;
  int rows = relax_res_rows();
  if (rows <= 0) rows = n >= 511 ? 4 : 2;
  while (2 * relax_res_blocks(n, rows) > kMaxSlotBlocks) rows *= 2;
  F.rows = rows;
  F.slots = h->slots;
  if ((rc = hip_check(launch_relax_res(F, s), "relaxation + residual"))) return rc;
  // algorithmic bytes of the two ops (each input once, r once in the
  // relaxation), one launch
  h->bytes += pts(rin) * sz(rin) + pts(L.y) * sz(L.y);
  h->bytes += pts(L.y) * sz(L.y) + pts(rin) * sz(rin) + pts(L.s) * sz(L.s);
  h->launches += 1;
  *done = true;
  return BFP_OK;
}

// y = V(l, rin)
int vcycle(mg_hierarchy* h, int l, const bfp_vec& rin, hipStream_t s) {
  Level& L = h->lv[l];
  const mg_params& p = h->prm;
  int rc;
  if (!recording() && l == h->Lc && h->prog[kPV].count && rin.mant == L.vr.mant &&
      rin.meta == L.vr.meta)
    return run_program(h, h->prog[kPV], s);
  // relaxation from y = 0: y = c2 A r + c1 r; with one pre-smoothing step
  // on a launched 2D level, optionally fused with the residual after it
  // when both are nnqcomp (their exponents follow from r's metadata alone)
  bool fused = false;
  if (l > 1 && p.nu1 == 1 && p.ndim == 2 && fuse_relax_res() && !recording() && !h->diag &&
      h->slots && mode_for(h, kRelax, false) == BFP_SATURATE &&
      mode_for(h, kVRes, false) == BFP_SATURATE) {
    if ((rc = relax_res(h, l, rin, s, &fused))) return rc;
  }
  if (!fused &&
      (rc = op_stencil(h, &h->A, rin, &p.c2, &p.c1, &rin, L.y, kRelax, mode_for(h, kRelax, false),
                       g_norm(rin, p.c1), s)))
    return rc;
  const bfp_vec* last = nullptr;
  for (int k = 1; k < p.nu1; ++k) {
    if ((rc = op_stencil(h, &h->A, L.y, &kOne, &kMinusOne, &rin, L.s,
                         kVRes, mode_for(h, kVRes, false), g_norm(rin, h->vres), s)))
      return rc;
    if ((rc = op_stencil(h, &h->A, L.s, &p.c2, &p.c1, &L.s, L.t, kRelax, mode_for(h, kRelax, false),
                         g_norm(L.s, p.c1), s)))
      return rc;
    if ((rc = op_sub(h, L.y, L.t, L.y, kVCorr, mode_for(h, kVCorr, false), g_sum(L.y, L.t), s)))
      return rc;
    last = &L.s;
  }
  if (l > 1) {
    Level& C = h->lv[l - 1];
    if (!fused && (rc = op_stencil(h, &h->A, L.y, &kOne, &kMinusOne, &rin, L.s,
                                   kVRes, mode_for(h, kVRes, false), g_norm(rin, h->vres), s)))
      return rc;
    if ((rc = op_stencil(h, &h->R, L.s, &kOne, nullptr, nullptr, C.vr,
                         kRestrict, mode_for(h, kRestrict, false), g_norm(L.s, kFour), s)))
      return rc;
    if ((rc = vcycle(h, l - 1, C.vr, s))) return rc;
    if ((rc = op_stencil(h, &h->P, C.y, &kMinusOne, &kOne, &L.y, L.y,
                         kVCorr, mode_for(h, kVCorr, false), g_sum(L.y, C.y), s)))
      return rc;
    last = &L.s;
  }
  for (int k = 0; k < p.nu2; ++k) {
    bfp_gamma g = last ? g_norm(*last, kOne) : g_norm(rin, h->vres);
    if ((rc = op_stencil(h, &h->A, L.y, &kOne, &kMinusOne, &rin, L.s,
                         kVRes, mode_for(h, kVRes, false), g, s)))
      return rc;
    if ((rc = op_stencil(h, &h->A, L.s, &p.c2, &p.c1, &L.s, L.t, kRelax, mode_for(h, kRelax, false),
                         g_norm(L.s, p.c1), s)))
      return rc;
    if ((rc = op_sub(h, L.y, L.t, L.y, kVCorr, mode_for(h, kVCorr, false), g_sum(L.y, L.t), s)))
      return rc;
    last = &L.s;
  }
  return BFP_OK;
}

// one IR-V iteration on level l; gamma = the estimate for the residual
// (force_q: the IR residual in qcomp whatever the policy)
int ir_iteration(mg_hierarchy* h, int l, const bfp_gamma* gres, bool first, bool plain_first2,
                 hipStream_t s, bool force_q = false) {
  Level& L = h->lv[l];
  int rc;
  const Site site = first ? kIrResFirst : kIrRes;
  int mode = mode_for(h, site, plain_first2);
  if (!gres || force_q) mode = BFP_NORMALIZE;   // no estimate exists, or forced: qcomp
  bfp_gamma gdummy{};
  gdummy.rule = BFP_GAMMA_EXPLICIT;
  if ((rc = op_stencil(h, &h->A, L.x, &kOne, &kMinusOne, &L.b, L.r, site, mode,
                       gres ? *gres : gdummy, s)))
    return rc;
  if ((rc = vcycle(h, l, L.r, s))) return rc;
  return op_sub(h, L.x, L.y, L.x, kIrCorr, mode_for(h, kIrCorr, false), g_sum(L.x, L.y), s);
}

// FMG levels lo..hi (lo = 1 starts from x_1 = 0)
int fmg_levels(mg_hierarchy* h, int lo, int hi, hipStream_t s) {
  const mg_params& p = h->prm;
  int rc;
  if (lo == 1) {
    if ((rc = bfp_vec_init(&h->lv[1].x, s))) return rc;
    h->launches += 2;
  }
  for (int l = lo; l <= hi; ++l) {
    Level& L = h->lv[l];
    if (l > 1) {
      Level& C = h->lv[l - 1];
      if ((rc = op_stencil(h, &h->P, C.x, &kOne, nullptr, nullptr, L.x,
                           kFmgProl, mode_for(h, kFmgProl, false), g_norm(C.x, kOne), s)))
        return rc;
    }
    for (int i = 1; i <= p.N; ++i) {
      bfp_gamma g = i > 1 ? g_norm(L.r, kOne)
                          : (l > 1 ? g_norm(h->lv[l - 1].r, kOne) : g_norm(L.b, kOne));
      if ((rc = ir_iteration(h, l, &g, i == 1, false, s))) return rc;
    }
  }
  return BFP_OK;
}

// levels whose grids fit the coarse-level executor
int exec_levels(const mg_params* p, int64_t maxp) {
  int lc = 0;
  for (int j = 1; j <= p->L; ++j) {
    const int64_t n = ((int64_t)1 << j) - 1;
    const int64_t pts = p->ndim == 3 ? n * n * n : n * n;
    if (pts > maxp || n >= kExecMaxN) break;
    lc = j;
  }
  return lc;
}

// Record the coarse-level programs of a laid-out hierarchy (no device work):
// the V-cycle on level Lc from vr, FMG on levels 1..Lc, the first, second
// and any later IR-V iteration on level Lc, and FMG on levels 1..Lc after
// quantizing b_1..b_Lc from FP64 (each conversion the bfp_vec_from_f64 that
// mg_set_rhs issues), through the same code that otherwise launches each
// operation.
int record_programs(mg_hierarchy* h, std::vector<ExecOp> (&P)[kPrograms],
                    double (&bytes)[kPrograms]) {
  for (int k = 0; k < kPrograms; ++k) {
    P[k].clear();
    bytes[k] = 0;
  }
  if (h->Lc == 0) return BFP_OK;
  const double b0 = h->bytes;
  const int64_t l0 = h->launches;
  const int Lc = h->Lc;
  Level& L = h->lv[Lc];
  int rc = BFP_OK;
  for (int k = 0; k < kPrograms && !rc; ++k) {
    const double before = h->bytes;
    record_into(&P[k]);
    if (k == kPV) {
      rc = vcycle(h, Lc, L.vr, nullptr);
    } else if (k == kPF) {
      rc = fmg_levels(h, 1, Lc, nullptr);
    } else if (k == kPFc) {
      for (int j = 1; j <= Lc; ++j) {
        const bfp_vec& b = h->lv[j].b;
        ExecOp e;
        std::memset(&e, 0, sizeof e);
        e.kind = kExConv;
        e.u.conv = ConvOp{nullptr, b.mant, b.meta, b.ndim, b.n, b.pitch, b.storage_bits, b.w,
                          rhs_shift(h->prm.ndim, j), j};
        P[k].push_back(e);
      }
      rc = fmg_levels(h, 1, Lc, nullptr);
    } else {
      // the i-th IR-V iteration on level Lc as mg_ir issues it (i = 1, 2, >2)
      const int i = k - kPI1 + 1;
      bfp_gamma g = g_norm(L.r, kOne);
      const bool plain_first2 = h->prm.policy == MG_POLICY_NN_IR_FIRST2_Q && i <= 2;
      rc = ir_iteration(h, Lc, i == 1 ? nullptr : &g, i == 1, plain_first2, nullptr);
    }
    record_into(nullptr);
    bytes[k] = h->bytes - before;
  }
  h->bytes = b0;
  h->launches = l0;
  return rc;
}

int check_params(const mg_params* p) {
  if (!p) return fail(BFP_EINVAL, "params are NULL");
  if (p->ndim != 2 && p->ndim != 3) return fail(BFP_ESHAPE, "ndim must be 2 or 3");
  if (p->L < 1 || p->L > MG_MAX_LEVELS) return fail(BFP_ESHAPE, "L must be in 1..%d", MG_MAX_LEVELS);
  if (p->nu1 < 1 || p->nu2 < 0 || p->N < 1) return fail(BFP_EINVAL, "need nu1 >= 1, nu2 >= 0, N >= 1");
  if (p->policy < MG_POLICY_Q || p->policy > MG_POLICY_NN_IR_Q) return fail(BFP_EINVAL, "bad policy");
  if (p->min_storage_bits != 0 && p->min_storage_bits != 8 && p->min_storage_bits != 16 &&
      p->min_storage_bits != 32)
    return fail(BFP_EWIDTH, "min_storage_bits must be 0, 8, 16 or 32");
  for (int j = 1; j <= p->L; ++j) {
    if (p->w_check[j] < 1 || p->w_check[j] > 32 || p->w_work[j] < 1 || p->w_work[j] > 32 ||
        p->w_inner[j] < 1 || p->w_inner[j] > 32)
      return fail(BFP_EWIDTH, "level %d: widths must be in 1..32", j);
  }
  if (p->c1.m <= 0 || p->c2.m >= 0) return fail(BFP_EINVAL, "need c1 > 0 > c2");
  if (p->c1.m >= (1 << 23) || p->c2.m < -(1 << 23) || p->c1_gamma.m <= 0 ||
      p->c1_gamma.m >= (1 << 23))
    return fail(BFP_EWIDTH, "Chebyshev coefficients must fit 24 bits");
  return BFP_OK;
}

// Lay out (or only size) every level's blocks in the arena, followed by
// room for `nops` recorded operations.
// diag: also reserve the diagnostic counters (h->diag) after the programs
size_t layout(mg_hierarchy* h, const mg_params* p, char* base, size_t nops, bool diag,
              bool slots = true) {
  size_t off = 0;
  const int mb = p->min_storage_bits;
  for (int j = 1; j <= p->L; ++j) {
    Level& L = h->lv[j];
    L.j = j;
    L.n = ((int64_t)1 << j) - 1;
    const int w_vr = j < p->L ? p->w_inner[j + 1] : p->w_inner[j];
    struct Spec { bfp_vec* v; int w; } specs[] = {
        {&L.x, p->w_work[j]}, {&L.b, p->w_check[j]}, {&L.r, p->w_inner[j]},
        {&L.vr, w_vr},        {&L.y, p->w_inner[j]}, {&L.s, p->w_inner[j]},
        {&L.t, p->w_inner[j]}};
    for (auto& sp : specs) {
      bfp_vec& v = *sp.v;
      v.w = sp.w;
      v.storage_bits = storage_for(sp.w, mb);
      v.ndim = p->ndim;
      v.n = (int32_t)L.n;
      v.pitch = pitch_for(L.n, v.storage_bits);
      const size_t bytes = (size_t)(v.pitch * rows_for(p->ndim, L.n) * (v.storage_bits / 8));
      v.mant = base ? base + off : nullptr;
      off = align256(off + bytes);
      v.meta = base ? (int64_t*)(base + off) : nullptr;
      off = align256(off + kMetaSlots * sizeof(int64_t));
    }
  }
  for (int k = 0; k < kPrograms; ++k)
    h->prog[k].metas = base ? (int64_t**)(base + off) + k * kExecMaxMeta : nullptr;
  off = align256(off + kPrograms * kExecMaxMeta * sizeof(int64_t*));
  h->prog[0].ops = base ? (ExecOp*)(base + off) : nullptr;
  off = align256(off + nops * sizeof(ExecOp));
  h->diag = nullptr;
  if (diag) {
    h->diag = base ? (int64_t*)(base + off) : nullptr;
    off = align256(off + kDiagBytes);
  }
  h->slots = nullptr;
  if (slots) {
    h->slots = base ? (int64_t*)(base + off) : nullptr;
    off = align256(off + 2 * (size_t)kMaxSlotBlocks * sizeof(int64_t));
  }
  return off;
}

// Host-side set-up shared by sizing and creation: stencils, the exact
// (2 c1 + 1) / 4, the executor levels.
int setup(mg_hierarchy* h, const mg_params* prm, int64_t exec_points) {
  h->prm = *prm;
  make_stencils(prm->ndim, &h->A, &h->R, &h->P);
  // (2 c1 + 1) / 4 exactly: c1 = m 2^e
  const bfp_scalar c = prm->c1_gamma;
  if (c.exp + 1 >= 0) {
    h->vres.m = (c.m << (c.exp + 1)) + 1;
    h->vres.exp = -2;
  } else {
    h->vres.m = c.m + ((int64_t)1 << (-(c.exp + 1)));
    h->vres.exp = c.exp - 1;
  }
  h->vres.w = 24;
  while (h->vres.m % 2 == 0) { h->vres.m /= 2; h->vres.exp += 1; }
  if (h->vres.m >= (1 << 23)) return fail(BFP_EWIDTH, "(2 c1 + 1) / 4 needs more than 24 bits");
  h->Lc = exec_levels(prm, exec_points);
  return BFP_OK;
}

// Number of recorded operations the hierarchy's programs hold: recorded
// on a layout at a stand-in address, with no device work.
int count_ops(const mg_params* prm, int64_t exec_points, size_t* nops) {
  mg_hierarchy* h = new (std::nothrow) mg_hierarchy();
  if (!h) return fail(BFP_ENOMEM, "host allocation failed");
  int rc = setup(h, prm, exec_points);
  if (!rc) {
    layout(h, prm, reinterpret_cast<char*>((uintptr_t)1 << 20), 0, false);
    std::vector<ExecOp> Pg[kPrograms];
    double bytes[kPrograms];
    rc = record_programs(h, Pg, bytes);
    *nops = 0;
    for (auto& v : Pg) *nops += v.size();
  }
  delete h;
  return rc;
}

// ------------------------------------------------------------ batches ---
//
// A batch holds many independent problems, each with its own hierarchy in
// the batch arena. Problems with identical parameters share one recorded,
// relocatable program: the conversion of the right-hand side on every level
// followed by the whole FMG, with every data and metadata pointer stored as
// an offset from the problem's arena base. One launch runs every problem's
// program, one workgroup per problem.

constexpr uintptr_t kStandIn = (uintptr_t)1 << 20;   // recording base of a program

struct BatchGroup {
  mg_params prm;
  mg_hierarchy* h;              // laid out at kStandIn
  std::vector<ExecOp> ops;      // relocated
  std::vector<int64_t*> metas;  // relocated
  size_t region;                // bytes of one problem's hierarchy
  double bytes;                 // algorithmic bytes of one solve
};

template <typename P>
void unbase(P*& p) {
  if (p) p = (P*)((uintptr_t)p - kStandIn);
}

int record_batch_program(BatchGroup& g) {
  mg_hierarchy* h = g.h;
  const mg_params& p = g.prm;
  g.ops.clear();
  const double b0 = h->bytes;
  for (int j = 1; j <= p.L; ++j) {
    const bfp_vec& b = h->lv[j].b;
    ExecOp e;
    std::memset(&e, 0, sizeof e);
    e.kind = kExConv;
    e.u.conv = ConvOp{nullptr, b.mant, b.meta, b.ndim, b.n, b.pitch, b.storage_bits, b.w,
                      rhs_shift(p.ndim, j), j};
    g.ops.push_back(e);
    h->bytes += pts(b) * (8.0 + sz(b));
  }
  record_into(&g.ops);
  int rc = fmg_levels(h, 1, p.L, nullptr);
  record_into(nullptr);
  g.bytes = h->bytes - b0;
  h->bytes = b0;
  if (rc) return rc;
  if ((rc = exec_assign_slots(g.ops, g.metas))) return rc;
  for (ExecOp& e : g.ops) {
    // relocatable programs keep no diagnostics (their pointers would not move)
    const OpArgs* a = e.kind == kExStar ? &e.u.star.op
                      : e.kind == kExTransfer ? &e.u.tr.op
                      : e.kind == kExPoint ? &e.u.pt.op : nullptr;
    if (a && a->diag) return fail(BFP_EINVAL, "batched program with diagnostics");
    switch (e.kind) {
      case kExStar: unbase(e.u.star.x); unbase(e.u.star.y); unbase(e.u.star.z); break;
      case kExTransfer: unbase(e.u.tr.x); unbase(e.u.tr.y); unbase(e.u.tr.z); break;
      case kExPoint: unbase(e.u.pt.x); unbase(e.u.pt.y); unbase(e.u.pt.z); break;
      case kExZero: unbase(e.u.zero.mant); break;
      case kExConv: unbase(e.u.conv.mant); break;
    }
  }
  for (int64_t*& m : g.metas) unbase(m);
  return BFP_OK;
}

}  // namespace

struct mg_batch {
  int nprob = 0, ndim = 0;
  std::vector<BatchGroup> groups;
  std::vector<int> group_of;        // per problem
  std::vector<uintptr_t> base;      // per problem
  BatchEntry* entries = nullptr;    // device, in launch order
  ExecOp* ops = nullptr;            // device
  int64_t** metas = nullptr;        // device
  double bytes = 0;                 // algorithmic bytes of one batched solve
  int64_t launches = 0;
  ~mg_batch() {
    for (BatchGroup& g : groups) delete g.h;
  }
};

namespace {

// Plan a batch: groups, programs, and the arena layout (base = null: sizes only).
int plan_batch(mg_batch* B, const mg_params* prms, int nprob, char* arena, size_t* total) {
  if (!prms || nprob < 1) return fail(BFP_EINVAL, "need at least one problem");
  B->nprob = nprob;
  B->ndim = prms[0].ndim;
  for (BatchGroup& g : B->groups) delete g.h;
  B->groups.clear();
  B->group_of.assign(nprob, -1);
  for (int i = 0; i < nprob; ++i) {
    int rc = check_params(&prms[i]);
    if (rc) return rc;
    if (prms[i].ndim != B->ndim) return fail(BFP_ESHAPE, "every problem of a batch needs the same ndim");
    const int64_t n = ((int64_t)1 << prms[i].L) - 1;
    if (n >= kExecMaxN) return fail(BFP_ESHAPE, "problem %d: batched grids need n < %d", i, kExecMaxN);
    int gi = -1;
    for (size_t k = 0; k < B->groups.size(); ++k)
      if (!std::memcmp(&B->groups[k].prm, &prms[i], sizeof(mg_params))) { gi = (int)k; break; }
    if (gi < 0) {
      BatchGroup g;
      g.prm = prms[i];
      g.h = new (std::nothrow) mg_hierarchy();
      if (!g.h) return fail(BFP_ENOMEM, "host allocation failed");
      B->groups.push_back(g);
      gi = (int)B->groups.size() - 1;
      BatchGroup& G = B->groups.back();
      if ((rc = setup(G.h, &G.prm, 0))) return rc;
      G.h->Lc = 0;
      G.region = layout(G.h, &G.prm, reinterpret_cast<char*>(kStandIn), 0, false, false);
      if ((rc = record_batch_program(G))) return rc;
    }
    B->group_of[i] = gi;
  }
  size_t off = 0;
  const size_t ent = align256(nprob * sizeof(BatchEntry));
  size_t nops = 0, nmeta = 0;
  for (BatchGroup& g : B->groups) { nops += g.ops.size(); nmeta += g.metas.size(); }
  B->entries = arena ? (BatchEntry*)(arena + off) : nullptr;
  off += ent;
  B->metas = arena ? (int64_t**)(arena + off) : nullptr;
  off = align256(off + nmeta * sizeof(int64_t*));
  B->ops = arena ? (ExecOp*)(arena + off) : nullptr;
  off = align256(off + nops * sizeof(ExecOp));
  B->base.assign(nprob, 0);
  B->bytes = 0;
  for (int i = 0; i < nprob; ++i) {
    B->base[i] = arena ? (uintptr_t)(arena + off) : 0;
    off = align256(off + B->groups[B->group_of[i]].region);
    B->bytes += B->groups[B->group_of[i]].bytes;
  }
  *total = off;
  return BFP_OK;
}

}  // namespace

extern "C" {

int bfp_cheby_coeffs(int64_t rho_num, int64_t rho_den, int64_t eta_num, int64_t eta_den,
                     int64_t scale_num, int64_t scale_den, int w, bfp_scalar* c1,
                     bfp_scalar* c2) {
  if (!c1 || !c2) return fail(BFP_EINVAL, "outputs are NULL");
  const int64_t lim = 1 << 12;
  if (rho_num <= 0 || rho_den <= 0 || eta_num <= 0 || eta_den <= eta_num || scale_num <= 0 ||
      scale_den <= 0 || rho_num > lim || rho_den > lim || eta_den > lim || scale_num > lim ||
      scale_den > lim)
    return fail(BFP_EINVAL, "need 0 < eta < 1, rho > 0, scale > 0 with terms up to 2^12");
  if (w < 2 || w > 24) return fail(BFP_EWIDTH, "w must be in 2..24");
  typedef __int128 i128;
  // alpha = An / Ad and c = Cn / Ad share a denominator; beta = den / (2 An Ad)
  const i128 An = (i128)(eta_den + eta_num) * rho_num, Cn = (i128)(eta_den - eta_num) * rho_num;
  const i128 Ad = (i128)2 * eta_den * rho_den;
  const i128 den = 2 * An * An - Cn * Cn;
  // c1 = 2 / beta = 4 An Ad / den, c2 = -1 / (alpha beta) = -2 Ad^2 / den, then rescaled
  const i128 q[2][2] = {{4 * An * Ad * scale_num, den * scale_den},
                        {-2 * Ad * Ad * scale_num * scale_num, den * scale_den * scale_den}};
  bfp_scalar* out[2] = {c1, c2};
  auto bitlen = [](i128 v) { int b = 0; while (v > 0) { ++b; v >>= 1; } return b; };
  for (int k = 0; k < 2; ++k) {
    const bool neg = (q[k][0] < 0) != (q[k][1] < 0);
    const i128 N = q[k][0] < 0 ? -q[k][0] : q[k][0];
    const i128 D = q[k][1] < 0 ? -q[k][1] : q[k][1];
    // fl = floor(log2(N / D)): the largest fl with D 2^fl <= N
    auto le = [&](int f) { return f >= 0 ? (D << f) <= N : D <= (N << -f); };
    int fl = bitlen(N) - bitlen(D) - 1;
    while (!le(fl)) --fl;
    while (le(fl + 1)) ++fl;
    // nu = floor(log2 q) + 2 for q > 0; for q < 0 it is ceil(log2 |q|) + 1
    const bool pow2 = fl >= 0 ? (D << fl) == N : D == (N << -fl);
    const int nu = neg ? (pow2 ? fl + 1 : fl + 2) : fl + 2;
    const int e = nu - w;
    i128 num = N, dd = D;
    if (e <= 0) num <<= -e; else dd <<= e;
    i128 m = num / dd;                        // floor of |q| / 2^e
    if (neg) m = (num % dd) ? -(m + 1) : -m;  // floor of a negative quotient
    out[k]->m = (int64_t)m;
    out[k]->exp = e;
    out[k]->w = w;
  }
  return BFP_OK;
}

int mg_params_init(int ndim, int L, int w, int progressive, int nu1, int nu2, int N,
                   int policy, int eta_percent, mg_params* out) {
  if (!out) return fail(BFP_EINVAL, "out is NULL");
  if (ndim != 2 && ndim != 3) return fail(BFP_ESHAPE, "ndim must be 2 or 3");
  if (L < 1 || L > MG_MAX_LEVELS) return fail(BFP_ESHAPE, "L must be in 1..%d", MG_MAX_LEVELS);
  if (w < 1 || w > 32) return fail(BFP_EWIDTH, "w must be in 1..32");
  if (eta_percent < 1 || eta_percent > 99) return fail(BFP_EINVAL, "eta_percent must be in 1..99");
  std::memset(out, 0, sizeof *out);
  out->ndim = ndim;
  out->L = L;
  out->nu1 = nu1;
  out->nu2 = nu2;
  out->N = N;
  out->policy = policy;
  for (int j = 1; j <= L; ++j) {
    if (!progressive) {
      out->w_check[j] = out->w_work[j] = out->w_inner[j] = w;
    } else {
      const int work = 2 * j + 8 < 32 ? 2 * j + 8 : 32;
      int inner = w - (L - j);
      if (inner < 5) inner = 5;
      if (inner > work) inner = work;
      out->w_check[j] = 32;
      out->w_work[j] = work;
      out->w_inner[j] = inner;
    }
  }
  int rc = bfpk::set_smoother(out, eta_percent);
  if (rc) return rc;
  return check_params(out);
}

}  // extern "C"

int bfpk::set_smoother(mg_params* p, int eta_percent) {
  if (eta_percent < 1 || eta_percent > 99) return fail(BFP_EINVAL, "eta_percent must be in 1..99");
  const int ndim = p->ndim;
  // D^-1 A = A' / a_c with a_c = 1 (2D) or 3/4 (3D): c1' = c1 / a_c, c2' = c2 / a_c^2
  int rc = bfp_cheby_coeffs(2, 1, eta_percent, 100, ndim == 2 ? 1 : 4, ndim == 2 ? 1 : 3, 16,
                            &p->c1, &p->c2);
  if (rc) return rc;
  bfp_scalar c2u;
  return bfp_cheby_coeffs(2, 1, eta_percent, 100, 1, 1, 16, &p->c1_gamma, &c2u);
}

extern "C" {

size_t mg_hierarchy_bytes(const mg_params* prm) {
  size_t b = 0;
  return hierarchy_bytes_ex(prm, exec_max_points(), &b) ? 0 : b;
}

int mg_hierarchy_create(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                        mg_hierarchy** out) {
  return hierarchy_create_ex(prm, arena_dev, bytes, stream, exec_max_points(), out);
}

}  // extern "C"

int bfpk::hierarchy_bytes_ex(const mg_params* prm, int64_t exec_points, size_t* bytes) {
  int rc = check_params(prm);
  if (rc) return rc;
  size_t nops = 0;
  if ((rc = count_ops(prm, exec_points, &nops))) return rc;
  mg_hierarchy tmp;
  *bytes = layout(&tmp, prm, nullptr, nops, diagnostics_on());
  return BFP_OK;
}

int bfpk::hierarchy_create_ex(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                              int64_t exec_points, mg_hierarchy** out) {
  int rc = check_params(prm);
  if (rc) return rc;
  if (!out || !arena_dev) return fail(BFP_EINVAL, "NULL argument");
  if ((uintptr_t)arena_dev % 256) return fail(BFP_EINVAL, "arena must be 256-byte aligned");
  size_t nops = 0;
  if ((rc = count_ops(prm, exec_points, &nops))) return rc;
  mg_hierarchy* h = new (std::nothrow) mg_hierarchy();
  if (!h) return fail(BFP_ENOMEM, "host allocation failed");
  if ((rc = setup(h, prm, exec_points))) { delete h; return rc; }
  const bool diag = diagnostics_on();
  const size_t need = layout(h, prm, nullptr, nops, diag);
  if (bytes < need) {
    delete h;
    return fail(BFP_ENOMEM, "arena holds %zu bytes, the hierarchy needs %zu", bytes, need);
  }
  layout(h, prm, static_cast<char*>(arena_dev), nops, diag);
  hipStream_t s = (hipStream_t)stream;
  for (int j = 1; j <= prm->L; ++j) {
    Level& L = h->lv[j];
    for (bfp_vec* v : {&L.x, &L.b, &L.r, &L.vr, &L.y, &L.s, &L.t}) {
      if ((rc = bfp_vec_init(v, stream))) { delete h; return rc; }
    }
  }
  if (h->diag && (rc = hip_check(hipMemsetAsync(h->diag, 0, kDiagBytes, s), "diagnostics reset"))) {
    delete h;
    return rc;
  }
  std::vector<ExecOp> Pg[kPrograms];
  std::vector<int64_t*> M[kPrograms];
  double pbytes[kPrograms];
  rc = record_programs(h, Pg, pbytes);
  for (int k = 0; k < kPrograms && !rc; ++k) rc = exec_assign_slots(Pg[k], M[k]);
  if (rc) {
    delete h;
    return rc;
  }
  std::vector<ExecOp> all;
  std::vector<int64_t*> tables(kPrograms * kExecMaxMeta, nullptr);
  for (int k = 0; k < kPrograms; ++k) {
    Program& pg = h->prog[k];
    pg.ops = h->prog[0].ops + all.size();
    pg.count = (int)Pg[k].size();
    pg.nmeta = (int)M[k].size();
    pg.bytes = pbytes[k];
    all.insert(all.end(), Pg[k].begin(), Pg[k].end());
    std::copy(M[k].begin(), M[k].end(), tables.begin() + k * kExecMaxMeta);
  }
  if (all.size() != nops) {
    delete h;
    return fail(BFP_EINVAL, "recorded programs changed size (%zu vs %zu ops)", all.size(), nops);
  }
  if (nops) {
    rc = hip_check(hipMemcpyAsync(h->prog[0].ops, all.data(), nops * sizeof(ExecOp),
                                  hipMemcpyHostToDevice, s), "program upload");
    if (!rc)
      rc = hip_check(hipMemcpyAsync(h->prog[0].metas, tables.data(), tables.size() * sizeof(int64_t*),
                                    hipMemcpyHostToDevice, s), "program upload");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "program upload");
    if (rc) { delete h; return rc; }
  }
  *out = h;
  return BFP_OK;
}

extern "C" {

int mg_hierarchy_destroy(mg_hierarchy* h) {
  delete h;
  return BFP_OK;
}

int mg_set_rhs(mg_hierarchy* h, int level, const double* f_dev, void* stream) {
  if (!h || level < 1 || level > h->prm.L) return fail(BFP_EINVAL, "bad level");
  const int64_t shift = rhs_shift(h->prm.ndim, level);
  return bfp_vec_from_f64(f_dev, shift, &h->lv[level].b, stream);
}

int mg_set_x(mg_hierarchy* h, int level, const double* x0_dev, void* stream) {
  if (!h || level < 1 || level > h->prm.L) return fail(BFP_EINVAL, "bad level");
  return bfp_vec_from_f64(x0_dev, 0, &h->lv[level].x, stream);
}

int mg_vcycle(mg_hierarchy* h, int level, const bfp_vec* r, bfp_vec* y, void* stream) {
  if (!h || level < 1 || level > h->prm.L || !r || !y) return fail(BFP_EINVAL, "bad argument");
  int rc = vcycle(h, level, *r, (hipStream_t)stream);
  if (rc) return rc;
  *y = h->lv[level].y;
  return BFP_OK;
}

int mg_ir(mg_hierarchy* h, int level, int iters, void* stream) {
  if (!h || level < 1 || level > h->prm.L || iters < 0) return fail(BFP_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  Level& L = h->lv[level];
  // level Lc: the recorded IR-V programs (first, second, later iterations)
  const bool progs = !recording() && level == h->Lc && h->prog[kPI1].count;
  for (int i = 1; i <= iters; ++i) {
    if (progs) {
      int rc = run_program(h, h->prog[kPI1 + std::min(i, 3) - 1], s);
      if (rc) return rc;
      continue;
    }
    bfp_gamma g = g_norm(L.r, kOne);
    const bool plain_first2 = h->prm.policy == MG_POLICY_NN_IR_FIRST2_Q && i <= 2;
    int rc = ir_iteration(h, level, i == 1 ? nullptr : &g, i == 1, plain_first2, s);
    if (rc) return rc;
  }
  return BFP_OK;
}

// exact: M 2^e > (num / 2^k) Mp 2^ep for M, Mp in [0, 2^31], num in [1, 2^31)
static bool norm_exceeds(int64_t M, int64_t e, int64_t Mp, int64_t ep, int64_t num, int k) {
  if (M == 0) return false;
  const unsigned __int128 B = (unsigned __int128)Mp * (uint64_t)num;   // < 2^62
  if (B == 0) return true;
  const int64_t d = e + k - ep;   // compare M 2^d with B
  if (d >= 64) return true;
  if (d <= -64) return false;
  if (d >= 0) return ((unsigned __int128)M << d) > B;
  return (unsigned __int128)M > (B << -d);
}

int mg_ir_safe(mg_hierarchy* h, int level, int iters, int q_iters, int32_t theta_num,
               int32_t theta_log2den, int* switched, void* stream) {
  if (!h || level < 1 || level > h->prm.L || iters < 0 || q_iters < 0)
    return fail(BFP_EINVAL, "bad argument");
  if (theta_num < 1 || theta_log2den < 0 || theta_log2den > 62)
    return fail(BFP_EINVAL, "theta must be num / 2^k with num >= 1 and 0 <= k <= 62");
  hipStream_t s = (hipStream_t)stream;
  Level& L = h->lv[level];
  int force = 0, nsw = 0, rc;
  bool have_prev = false;
  int64_t prevM = 0, preve = 0;
  int64_t meta[kExMetaF];
  for (int i = 1; i <= iters; ++i) {
    const bool fallback = force > 0;
    bfp_gamma g = g_norm(L.r, kOne);
    const bool plain_first2 = h->prm.policy == MG_POLICY_NN_IR_FIRST2_Q && i <= 2;
    if ((rc = ir_iteration(h, level, i == 1 ? nullptr : &g, i == 1, plain_first2, s, fallback)))
      return rc;
    if (fallback) {
      ++nsw;
      --force;
    }
    // the residual's saturations and norm decide the next iterations
    if ((rc = hip_check(hipMemcpyAsync(meta, L.r.meta, sizeof meta, hipMemcpyDeviceToHost, s),
                        "residual metadata")) ||
        (rc = hip_check(hipStreamSynchronize(s), "residual metadata")))
      return rc;
    const int64_t M = std::max(meta[kMetaMax], -meta[kMetaMin]);
    if (meta[kMetaSat] > 0 ||
        (have_prev && norm_exceeds(M, meta[kMetaExp], prevM, preve, theta_num, theta_log2den)))
      force = q_iters;
    have_prev = true;
    prevM = M;
    preve = meta[kMetaExp];
  }
  if (switched) *switched = nsw;
  return BFP_OK;
}

int mg_fmg(mg_hierarchy* h, void* stream) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  hipStream_t s = (hipStream_t)stream;
  int rc;
  int lo = 1;
  if (h->prog[kPF].count) {
    if ((rc = run_program(h, h->prog[kPF], s))) return rc;
    lo = h->Lc + 1;
  }
  return fmg_levels(h, lo, h->prm.L, s);
}

int mg_fmg_f64(mg_hierarchy* h, const double* const* rhs_dev, void* stream) {
  if (!h || !rhs_dev) return fail(BFP_EINVAL, "NULL argument");
  const int L = h->prm.L, Lc = h->Lc;
  for (int j = 1; j <= L; ++j)
    if (!rhs_dev[j - 1]) return fail(BFP_EINVAL, "right-hand side of level %d is NULL", j);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  const Program& pc = h->prog[kPFc];
  if (!pc.count) {   // no executor levels: quantize every level, then FMG
    for (int j = 1; j <= L; ++j)
      if ((rc = mg_set_rhs(h, j, rhs_dev[j - 1], stream))) return rc;
    return mg_fmg(h, stream);
  }
  if (Lc < L) {
    // levels Lc+1..L are quantized on the side stream, after everything
    // issued on `stream` so far, while the program runs levels 1..Lc
    if (!h->side) {
      if ((rc = hip_check(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking), "side stream")) ||
          (rc = hip_check(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming), "event")) ||
          (rc = hip_check(hipEventCreateWithFlags(&h->join, hipEventDisableTiming), "event")))
        return rc;
    }
    if ((rc = hip_check(hipEventRecord(h->fork, s), "event record")) ||
        (rc = hip_check(hipStreamWaitEvent(h->side, h->fork, 0), "stream wait")))
      return rc;
    for (int j = Lc + 1; j <= L; ++j)
      if ((rc = mg_set_rhs(h, j, rhs_dev[j - 1], h->side))) return rc;
    if ((rc = hip_check(hipEventRecord(h->join, h->side), "event record"))) return rc;
  }
  ExecRhs r{};
  for (int j = 1; j <= L; ++j) r.p[j - 1] = rhs_dev[j - 1];
  if ((rc = run_program(h, pc, s, &r))) return rc;
  if (Lc < L && (rc = hip_check(hipStreamWaitEvent(s, h->join, 0), "stream wait"))) return rc;
  return fmg_levels(h, Lc + 1, L, s);
}

}  // extern "C"

// mg_fmg_f64 with every step on `stream` (no second stream): the finer
// levels' right-hand sides are quantized before the coarse-level program
// runs. The same blocks as mg_fmg_f64.
int bfpk::fmg_f64_one_stream(mg_hierarchy* h, const double* const* rhs_dev, hipStream_t s) {
  if (!h || !rhs_dev) return fail(BFP_EINVAL, "NULL argument");
  const int L = h->prm.L, Lc = h->Lc;
  for (int j = 1; j <= L; ++j)
    if (!rhs_dev[j - 1]) return fail(BFP_EINVAL, "right-hand side of level %d is NULL", j);
  int rc;
  const Program& pc = h->prog[kPFc];
  if (!pc.count) {
    for (int j = 1; j <= L; ++j)
      if ((rc = mg_set_rhs(h, j, rhs_dev[j - 1], s))) return rc;
    return mg_fmg(h, s);
  }
  for (int j = Lc + 1; j <= L; ++j)
    if ((rc = mg_set_rhs(h, j, rhs_dev[j - 1], s))) return rc;
  ExecRhs r{};
  for (int j = 1; j <= L; ++j) r.p[j - 1] = rhs_dev[j - 1];
  if ((rc = run_program(h, pc, s, &r))) return rc;
  return fmg_levels(h, Lc + 1, L, s);
}

extern "C" {

int mg_autotune(mg_hierarchy* h, int reps, void* stream, mg_tune_report* out) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  if (reps < 1 || reps > 1000) return fail(BFP_EINVAL, "reps must be in 1..1000");
  hipStream_t s = (hipStream_t)stream;
  const int nd = h->prm.ndim, L = h->prm.L;
  const double b0 = h->bytes;
  const int64_t l0 = h->launches;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_check(hipEventCreate(&e0), "event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "event");
  mg_tune_report rep;
  std::memset(&rep, 0, sizeof rep);
  rep.first_level = h->Lc + 1;
  rep.last_level = L;
  // average time of `reps` back-to-back launches of op(), median of three
  auto timed = [&](auto op, float* us) {
    float t[3];
    for (int k = 0; k < 3 && !rc; ++k) {
      for (int i = 0; i < 2 && !rc; ++i) rc = op();
      if (!rc) rc = hip_check(hipEventRecord(e0, s), "event record");
      for (int i = 0; i < reps && !rc; ++i) rc = op();
      if (!rc) rc = hip_check(hipEventRecord(e1, s), "event record");
      if (!rc) rc = hip_check(hipEventSynchronize(e1), "event sync");
      float ms = 0;
      if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
      t[k] = ms * 1000.0f / reps;
    }
    if (rc) return;
    std::sort(t, t + 3);
    *us = t[1];
  };
  const int cands[] = {1, 2, 4, 8, 16, 32, 64};
  for (int j = h->Lc + 1; j <= L && !rc; ++j) {
    Level& V = h->lv[j];
    // the IR residual r = A x - b (the star kernel with a y stream)
    auto star = [&]() {
      return op_stencil(h, &h->A, V.x, &kOne, &kMinusOne, &V.b, V.r, kIrRes, BFP_SATURATE,
                        g_norm(V.r, kOne), s);
    };
    float best = 0, t = 0;
    int pick = 0;
    set_level_rows(0, nd, j, 0);
    timed(star, &rep.star_default_us[j]);
    for (int c : cands) {
      if (rc || c > V.n) break;
      set_level_rows(0, nd, j, c);
      timed(star, &t);
      if (!rc && (!pick || t < best)) { best = t; pick = c; }
    }
    if (rc) break;
    if (best < rep.star_default_us[j]) {
      set_level_rows(0, nd, j, pick);
      rep.star_rows[j] = pick;
      rep.star_us[j] = best;
    } else {
      set_level_rows(0, nd, j, 0);
      rep.star_us[j] = rep.star_default_us[j];
    }
    if (j < 2) continue;
    // restriction s_j -> vr_(j-1) and prolongation-correction t_j = y_j - P y_(j-1)
    Level& Cl = h->lv[j - 1];
    auto transfer = [&]() {
      int e = op_stencil(h, &h->R, V.s, &kOne, nullptr, nullptr, Cl.vr, kRestrict, BFP_SATURATE,
                         g_norm(V.s, kFour), s);
      if (e) return e;
      return op_stencil(h, &h->P, Cl.y, &kMinusOne, &kOne, &V.y, V.t, kVCorr, BFP_SATURATE,
                        g_sum(V.y, Cl.y), s);
    };
    best = 0;
    pick = 0;
    set_level_rows(1, nd, j, 0);
    timed(transfer, &rep.transfer_default_us[j]);
    for (int c : cands) {
      if (rc || c > 32 || c > Cl.n + 1) break;
      set_level_rows(1, nd, j, c);
      timed(transfer, &t);
      if (!rc && (!pick || t < best)) { best = t; pick = c; }
    }
    if (rc) break;
    if (best < rep.transfer_default_us[j]) {
      set_level_rows(1, nd, j, pick);
      rep.transfer_rows[j] = pick;
      rep.transfer_us[j] = best;
    } else {
      set_level_rows(1, nd, j, 0);
      rep.transfer_us[j] = rep.transfer_default_us[j];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->bytes = b0;
  h->launches = l0;
  if (!rc && out) *out = rep;
  return rc;
}

// Launch shapes chosen by the time of whole FMG solves: each level's star
// and transfer march lengths in turn (coordinate descent from the finest
// level down, the other levels at their current shapes), so every shape is
// judged in the conditions of the solve (caches, the executor's tails, the
// neighbouring launches) rather than by back-to-back launches of one op.
int mg_autotune_solve(mg_hierarchy* h, int reps, void* stream, mg_tune_report* out) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  if (reps < 1 || reps > 100) return fail(BFP_EINVAL, "reps must be in 1..100");
  hipStream_t s = (hipStream_t)stream;
  const int nd = h->prm.ndim, L = h->prm.L;
  const double b0 = h->bytes;
  const int64_t l0 = h->launches;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_check(hipEventCreate(&e0), "event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "event");
  mg_tune_report rep;
  std::memset(&rep, 0, sizeof rep);
  rep.first_level = h->Lc + 1;
  rep.last_level = L;
  // time of one FMG solve over one run of `reps` solves (after one more)
  auto timed1 = [&](float* us) {
    if (!rc) rc = mg_fmg(h, s);
    if (!rc) rc = hip_check(hipEventRecord(e0, s), "event record");
    for (int i = 0; i < reps && !rc; ++i) rc = mg_fmg(h, s);
    if (!rc) rc = hip_check(hipEventRecord(e1, s), "event record");
    if (!rc) rc = hip_check(hipEventSynchronize(e1), "event sync");
    float ms = 0;
    if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
    *us = ms * 1000.0f / reps;
  };
  auto median3 = [](float* t) {
    std::sort(t, t + 3);
    return t[1];
  };
  const int cands[] = {1, 2, 4, 8, 16, 32, 64};
  // one kind (0 star, 1 transfer) on level j: every candidate is timed in
  // turns with the incumbent (three runs each, medians compared), so a
  // drift of the clock during the search favours neither; a candidate
  // replaces the incumbent when at least 0.3% faster
  auto search = [&](int kind, int j, int maxc, int32_t* pick_out, float* best_out,
                    float* default_out) {
    int pick = 0;
    float best = 0;
    for (int c : cands) {
      if (rc || c > maxc) break;
      float ti[3], tc[3];
      for (int k = 0; k < 3 && !rc; ++k) {
        set_level_rows(kind, nd, j, pick);
        timed1(&ti[k]);
        set_level_rows(kind, nd, j, c);
        timed1(&tc[k]);
      }
      if (rc) break;
      const float mi = median3(ti), mc = median3(tc);
      if (pick == 0 && c == cands[0]) *default_out = mi;
      if (best == 0) best = mi;
      if (mc < mi * 0.997f) {
        pick = c;
        best = mc;
      } else {
        best = mi;
      }
    }
    if (rc) return;
    set_level_rows(kind, nd, j, pick);
    *pick_out = pick;
    *best_out = best;
  };
  for (int j = L; j > h->Lc && !rc; --j) {
    search(0, j, h->lv[j].n, &rep.star_rows[j], &rep.star_us[j], &rep.star_default_us[j]);
    if (!rc && j >= 2)
      search(1, j, std::min<int64_t>(32, h->lv[j - 1].n + 1), &rep.transfer_rows[j],
             &rep.transfer_us[j], &rep.transfer_default_us[j]);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->bytes = b0;
  h->launches = l0;
  if (!rc && out) *out = rep;
  return rc;
}

int mg_diag_read(mg_hierarchy* h, int64_t* host_out, int reset, void* stream) {
  if (!h || !host_out) return fail(BFP_EINVAL, "NULL argument");
  if (!h->diag)
    return fail(BFP_EINVAL, "this hierarchy keeps no diagnostics (created with tuning key "
                            "\"diagnostics\" = 0)");
  hipStream_t s = (hipStream_t)stream;
  int rc = hip_check(hipStreamSynchronize(s), "diagnostics read");
  if (!rc) rc = hip_check(hipMemcpy(host_out, h->diag, kDiagBytes, hipMemcpyDeviceToHost),
                          "diagnostics read");
  if (!rc && reset) {
    rc = hip_check(hipMemsetAsync(h->diag, 0, kDiagBytes, s), "diagnostics reset");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "diagnostics reset");
  }
  return rc;
}

int mg_get_vec(mg_hierarchy* h, int level, int which, bfp_vec* out) {
  if (!h || !out || level < 1 || level > h->prm.L) return fail(BFP_EINVAL, "bad argument");
  Level& L = h->lv[level];
  switch (which) {
    case 0: *out = L.x; return BFP_OK;
    case 1: *out = L.b; return BFP_OK;
    case 2: *out = L.r; return BFP_OK;
    case 3: *out = L.y; return BFP_OK;
  }
  return fail(BFP_EINVAL, "unknown block %d", which);
}

int mg_counters(const mg_hierarchy* h, double* bytes, int64_t* launches) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  if (bytes) *bytes = h->bytes;
  if (launches) *launches = h->launches;
  return BFP_OK;
}

size_t mg_batch_bytes(const mg_params* prms, int nprob) {
  mg_batch B;
  size_t total = 0;
  if (plan_batch(&B, prms, nprob, nullptr, &total)) return 0;
  return total;
}

int mg_batch_create(const mg_params* prms, int nprob, void* arena_dev, size_t bytes,
                    void* stream, mg_batch** out) {
  if (!out || !arena_dev) return fail(BFP_EINVAL, "NULL argument");
  if ((uintptr_t)arena_dev % 256) return fail(BFP_EINVAL, "arena must be 256-byte aligned");
  mg_batch* B = new (std::nothrow) mg_batch();
  if (!B) return fail(BFP_ENOMEM, "host allocation failed");
  size_t need = 0;
  int rc = plan_batch(B, prms, nprob, nullptr, &need);
  if (!rc && bytes < need)
    rc = fail(BFP_ENOMEM, "arena holds %zu bytes, the batch needs %zu", bytes, need);
  if (!rc) rc = plan_batch(B, prms, nprob, static_cast<char*>(arena_dev), &need);
  if (rc) { delete B; return rc; }
  hipStream_t s = (hipStream_t)stream;
  // device tables: entries (largest programs first), metadata tables, ops
  std::vector<ExecOp> ops;
  std::vector<int64_t*> metas;
  std::vector<int> op_begin(B->groups.size()), meta_begin(B->groups.size());
  for (size_t k = 0; k < B->groups.size(); ++k) {
    op_begin[k] = (int)ops.size();
    meta_begin[k] = (int)metas.size();
    ops.insert(ops.end(), B->groups[k].ops.begin(), B->groups[k].ops.end());
    metas.insert(metas.end(), B->groups[k].metas.begin(), B->groups[k].metas.end());
  }
  std::vector<BatchEntry> ent(nprob);
  for (int i = 0; i < nprob; ++i) {
    const int k = B->group_of[i];
    ent[i] = BatchEntry{B->base[i], i, op_begin[k], (int)B->groups[k].ops.size(), meta_begin[k],
                        (int)B->groups[k].metas.size()};
  }
  std::stable_sort(ent.begin(), ent.end(),
                   [](const BatchEntry& a, const BatchEntry& b) { return a.op_count > b.op_count; });
  // initial state: zero mantissas, metadata at exponent 1 - w with identities
  std::vector<int64_t*> mlist;
  std::vector<int64_t> elist;
  for (int i = 0; i < nprob; ++i) {
    const BatchGroup& g = B->groups[B->group_of[i]];
    for (int j = 1; j <= g.prm.L; ++j) {
      const Level& L = g.h->lv[j];
      for (const bfp_vec* v : {&L.x, &L.b, &L.r, &L.vr, &L.y, &L.s, &L.t}) {
        mlist.push_back((int64_t*)((uintptr_t)v->meta - kStandIn + B->base[i]));
        elist.push_back(1 - v->w);
      }
    }
  }
  char* first = (char*)B->base[0];
  const size_t region_bytes = (size_t)((char*)arena_dev + need - first);
  void* scratch = nullptr;
  const size_t lists = mlist.size() * (sizeof(int64_t*) + sizeof(int64_t));
  rc = hip_check(hipMemsetAsync(first, 0, region_bytes, s), "batch arena clear");
  if (!rc) rc = hip_check(hipMalloc(&scratch, lists), "batch set-up buffer");
  if (!rc) rc = hip_check(hipMemcpyAsync(scratch, mlist.data(), mlist.size() * sizeof(int64_t*),
                                         hipMemcpyHostToDevice, s), "batch set-up copy");
  int64_t* exps_dev = scratch ? (int64_t*)((char*)scratch + mlist.size() * sizeof(int64_t*)) : nullptr;
  if (!rc) rc = hip_check(hipMemcpyAsync(exps_dev, elist.data(), elist.size() * sizeof(int64_t),
                                         hipMemcpyHostToDevice, s), "batch set-up copy");
  if (!rc) rc = hip_check(launch_meta_init_list((int64_t* const*)scratch, exps_dev,
                                                (int)mlist.size(), s), "batch metadata init");
  if (!rc) rc = hip_check(hipMemcpyAsync(B->entries, ent.data(), ent.size() * sizeof(BatchEntry),
                                         hipMemcpyHostToDevice, s), "batch upload");
  if (!rc && !metas.empty())
    rc = hip_check(hipMemcpyAsync(B->metas, metas.data(), metas.size() * sizeof(int64_t*),
                                  hipMemcpyHostToDevice, s), "batch upload");
  if (!rc) rc = hip_check(hipMemcpyAsync(B->ops, ops.data(), ops.size() * sizeof(ExecOp),
                                         hipMemcpyHostToDevice, s), "batch upload");
  const int rs = hip_check(hipStreamSynchronize(s), "batch upload");
  if (!rc) rc = rs;
  if (scratch) hipFree(scratch);
  if (rc) { delete B; return rc; }
  *out = B;
  return BFP_OK;
}

int mg_batch_destroy(mg_batch* b) {
  delete b;
  return BFP_OK;
}

int mg_solve_batch(mg_batch* b, const double* const* rhs_table_dev, void* stream) {
  if (!b || !rhs_table_dev) return fail(BFP_EINVAL, "NULL argument");
  int rc = hip_check(launch_exec_batch(b->entries, b->nprob, b->ops, b->metas, rhs_table_dev,
                                       b->ndim, (hipStream_t)stream), "batched solve");
  if (rc) return rc;
  b->launches += 1;
  return BFP_OK;
}

int mg_batch_get_vec(mg_batch* b, int prob, int level, int which, bfp_vec* out) {
  if (!b || !out || prob < 0 || prob >= b->nprob) return fail(BFP_EINVAL, "bad argument");
  const BatchGroup& g = b->groups[b->group_of[prob]];
  if (level < 1 || level > g.prm.L) return fail(BFP_EINVAL, "bad level");
  const Level& L = g.h->lv[level];
  const bfp_vec* v = which == 0 ? &L.x : which == 1 ? &L.b : which == 2 ? &L.r : which == 3 ? &L.y : nullptr;
  if (!v) return fail(BFP_EINVAL, "unknown block %d", which);
  *out = *v;
  out->mant = (void*)((uintptr_t)v->mant - kStandIn + b->base[prob]);
  out->meta = (int64_t*)((uintptr_t)v->meta - kStandIn + b->base[prob]);
  return BFP_OK;
}

int mg_batch_counters(const mg_batch* b, double* bytes, int64_t* launches) {
  if (!b) return fail(BFP_EINVAL, "NULL batch");
  if (bytes) *bytes = b->bytes;
  if (launches) *launches = b->launches;
  return BFP_OK;
}

}  // extern "C"
static_assert(bfpk::kMaxLevels == MG_MAX_LEVELS, "right-hand-side table rows");

int bfpk::params_ok(const mg_params* p) { return check_params(p); }

int bfpk::set_rhs_table(mg_hierarchy* h, int level, const double* const* table_dev, int index,
                        hipStream_t s) {
  if (!h || level < 1 || level > h->prm.L) return fail(BFP_EINVAL, "bad level");
  const int64_t shift = rhs_shift(h->prm.ndim, level);
  return from_f64_impl(nullptr, table_dev, index, shift, &h->lv[level].b, s);
}
