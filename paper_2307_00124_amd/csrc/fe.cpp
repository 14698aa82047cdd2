// The paper's finite-element model problems (Section 6): 1D B-spline
// Rayleigh-Ritz discretizations of Poisson (m = 1) and the biharmonic
// equation (m = 2), solved by BFP FMG.
//
// Set-up S (Appendix C) is applied in exact rational arithmetic (128-bit
// numerators and denominators, reduced after every step) to the caller's
// reference stiffness matrices K_hat_j, prolongations P_j and FP64 load
// vectors F_hat_j (K_j = h^(1-2m) K_hat_j, F_j = h F_hat_j, D_j = diag K_j):
//   A_j = D_hat_j^-1 K_hat_j,  b_j = 2^(-2mj) F_hat_j / diag(K_hat_j),
//   R_j = 2^(2m-1) D_hat_(j-1)^-1 P_j^T D_hat_j.
// These operators are not dyadic, so every call site quantizes its operator
// on entry as Algorithms IR, V and FMG do: A at the check width for the IR
// residual, A, R and P at the inner width inside the V-cycle, P at the
// working width for the FMG prolongation (normalized floor quantization of
// the whole matrix, one exponent). rho for the Chebyshev coefficients is the
// Gershgorin bound of A on level min(5, L) (an upper bound of the largest
// generalized eigenvalue), eta = eta_num / eta_den; c1, c2 floor-quantized
// to 16 bits. Every operation is a qcomp (two passes); the banded products
// run in k_band.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"
#include "band.hpp"
#include "kernels.hpp"

using namespace bfpk;

namespace {

typedef __int128 i128;

i128 iabs(i128 v) { return v < 0 ? -v : v; }

i128 gcd128(i128 a, i128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b) {
    const i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

int bitlen(i128 v) {
  unsigned __int128 u = (unsigned __int128)iabs(v);
  int b = 0;
  while (u) {
    ++b;
    u >>= 1;
  }
  return b;
}

// An exact rational num / den (den > 0, reduced); ok = false once a step
// would not fit 128 bits.
struct Q {
  i128 n = 0, d = 1;
};

bool fits(i128 a, i128 b) { return bitlen(a) + bitlen(b) <= 125; }

bool make(i128 n, i128 d, Q* out) {
  if (d == 0) return false;
  if (d < 0) {
    n = -n;
    d = -d;
  }
  const i128 g = gcd128(n, d);
  if (g > 1) {
    n /= g;
    d /= g;
  }
  out->n = n;
  out->d = d;
  return true;
}

bool mul(const Q& a, const Q& b, Q* out) {
  // cross-reduce first
  const i128 g1 = gcd128(a.n, b.d), g2 = gcd128(b.n, a.d);
  const i128 an = g1 ? a.n / g1 : a.n, bd = g1 ? b.d / g1 : b.d;
  const i128 bn = g2 ? b.n / g2 : b.n, ad = g2 ? a.d / g2 : a.d;
  if (!fits(an, bn) || !fits(ad, bd)) return false;
  return make(an * bn, ad * bd, out);
}

bool divq(const Q& a, const Q& b, Q* out) {
  if (b.n == 0) return false;
  return mul(a, Q{b.d, b.n}, out) && make(out->n, out->d, out);
}

bool add(const Q& a, const Q& b, Q* out) {
  const i128 g = gcd128(a.d, b.d);
  const i128 da = a.d / g, db = b.d / g;
  if (!fits(a.n, db) || !fits(b.n, da) || !fits(a.d, db)) return false;
  return make(a.n * db + b.n * da, a.d * db, out);
}

bool mul_pow2(const Q& a, int k, Q* out) {
  if (k >= 0) {
    if (bitlen(a.n) + k > 125) return false;
    return make(a.n << k, a.d, out);
  }
  if (bitlen(a.d) - k > 125) return false;
  return make(a.n, a.d << (-k), out);
}

// nu(q) = the smallest b with -2^(b-1) <= q < 2^(b-1), q != 0
int nu_q(const Q& q) {
  const i128 A = iabs(q.n), B = q.d;
  // t = floor(log2(A / B))
  int t = bitlen(A) - bitlen(B);
  bool ge;   // A >= B 2^t
  if (t >= 0) ge = A >= (B << t);
  else ge = (A << (-t)) >= B;
  if (!ge) --t;
  if (q.n > 0) return t + 2;
  // negative: the smallest b with |q| <= 2^(b-1)
  const bool pow2 = t >= 0 ? A == (B << t) : (A << (-t)) == B;
  return t + 1 + (pow2 ? 0 : 1);
}

// floor(q / 2^e); saturates to 0 / -1 when the quotient is below 1 in
// magnitude beyond 128-bit reach
i128 floor_div_pow2(const Q& q, int e) {
  i128 n = q.n, d = q.d;
  if (e <= 0) {
    if (bitlen(n) - e > 125) return 0;   // not reached for normalized outputs
    n <<= (-e);
  } else {
    if (bitlen(d) + e > 125) return n >= 0 ? 0 : -1;
    d <<= e;
  }
  i128 r = n / d;
  if ((n % d) != 0 && n < 0) --r;
  return r;
}

// the FP64 value v as an exact rational
bool from_double(double v, Q* out) {
  if (v == 0) {
    *out = Q{0, 1};
    return true;
  }
  int ex = 0;
  const double f = frexp(v, &ex);   // v = f 2^ex, |f| in [0.5, 1)
  const int64_t z = (int64_t)ldexp(f, 53);
  Q q{z, 1};
  return mul_pow2(q, ex - 53, out);
}

struct RBand {   // a banded matrix of rationals (host)
  int nrows = 0, ncols = 0;
  std::vector<int> col0;
  std::vector<std::vector<Q>> v;
};

struct DevBand {   // a quantized banded matrix on the device
  int32_t* col0 = nullptr;
  int32_t* taps = nullptr;
  int64_t e = 0;
  int band = 0, nrows = 0, ncols = 0;
  int64_t rowabs = 0;   // largest sum |taps| of a row
};

struct FeVec {
  int32_t* mant = nullptr;
  int64_t* meta = nullptr;
  int n = 0;
  int w = 1;   // width of the mantissas it holds
};

}  // namespace

struct fe_hierarchy {
  fe_params prm;
  int n[MG_MAX_LEVELS + 1];
  DevBand A_check[MG_MAX_LEVELS + 1], A_inner[MG_MAX_LEVELS + 1], R_inner[MG_MAX_LEVELS + 1],
      P_inner[MG_MAX_LEVELS + 1], P_work[MG_MAX_LEVELS + 1];
  FeVec x[MG_MAX_LEVELS + 1], b[MG_MAX_LEVELS + 1], r[MG_MAX_LEVELS + 1], y[MG_MAX_LEVELS + 1],
      rv[MG_MAX_LEVELS + 1], vin[MG_MAX_LEVELS + 1];
  bfp_scalar c1{}, c2{};
  std::vector<void*> allocs;
  double bytes = 0;
  int64_t launches = 0;
  // the whole FMG recorded as one single-workgroup program (null when some
  // op does not fit one workgroup or recording failed)
  BandStep* prog = nullptr;
  int prog_steps = 0;
  double prog_bytes = 0;
  std::vector<BandStep>* rec = nullptr;   // set while recording
  bool rec_ok = true;
};

namespace {

int alloc(fe_hierarchy* h, size_t bytes, void** p) {
  int rc = hip_check(hipMalloc(p, bytes < 16 ? 16 : bytes), "hipMalloc");
  if (!rc) h->allocs.push_back(*p);
  return rc;
}

int band_from_input(const fe_rational_band* in, RBand* out) {
  if (!in || in->nrows < 1 || in->ncols < 1 || in->band < 1 || !in->col0 || !in->num || !in->den)
    return fail(BFP_EINVAL, "bad banded matrix");
  out->nrows = in->nrows;
  out->ncols = in->ncols;
  out->col0.assign(in->col0, in->col0 + in->nrows);
  out->v.assign(in->nrows, std::vector<Q>(in->band));
  for (int i = 0; i < in->nrows; ++i) {
    if (in->col0[i] < 0 || in->col0[i] + in->band > in->ncols)
      return fail(BFP_ESHAPE, "banded matrix row %d reaches outside its columns", i);
    for (int t = 0; t < in->band; ++t) {
      const int64_t d = in->den[(int64_t)i * in->band + t];
      if (d <= 0) return fail(BFP_EINVAL, "denominators must be positive");
      make(in->num[(int64_t)i * in->band + t], d, &out->v[i][t]);
    }
  }
  return BFP_OK;
}

// Q_w of a rational banded matrix, uploaded
int quantize_upload(fe_hierarchy* h, const RBand& B, int w, DevBand* out) {
  int numax = INT32_MIN;
  for (const auto& row : B.v)
    for (const Q& q : row)
      if (q.n != 0) numax = std::max(numax, nu_q(q));
  const int64_t e = numax == INT32_MIN ? 1 - w : (int64_t)numax - w;
  int band = 0;
  for (const auto& row : B.v) band = std::max(band, (int)row.size());
  band = std::min(band, B.ncols);
  // every row stores `band` taps from a column that keeps them inside the
  // input (zeros pad the row on the side that would fall outside)
  std::vector<int32_t> taps((size_t)B.nrows * band, 0), col0(B.nrows);
  int64_t rowabs = 0;
  for (int i = 0; i < B.nrows; ++i) {
    const int c = std::max(0, std::min(B.col0[i], B.ncols - band));
    col0[i] = c;
    int64_t s = 0;
    for (size_t t = 0; t < B.v[i].size(); ++t) {
      const i128 m = floor_div_pow2(B.v[i][t], (int)e);
      const int at = B.col0[i] + (int)t - c;
      if (m != 0 && (at < 0 || at >= band)) return fail(BFP_ESHAPE, "row %d is wider than the band", i);
      if (at >= 0 && at < band) taps[(size_t)i * band + at] = (int32_t)m;
      s += (int64_t)(m < 0 ? -m : m);
    }
    rowabs = std::max(rowabs, s);
  }
  out->e = e;
  out->band = band;
  out->nrows = B.nrows;
  out->ncols = B.ncols;
  out->rowabs = rowabs;
  int rc;
  if ((rc = alloc(h, taps.size() * 4, (void**)&out->taps))) return rc;
  if ((rc = alloc(h, col0.size() * 4, (void**)&out->col0))) return rc;
  if ((rc = hip_check(hipMemcpy(out->taps, taps.data(), taps.size() * 4, hipMemcpyHostToDevice),
                      "upload")))
    return rc;
  return hip_check(hipMemcpy(out->col0, col0.data(), col0.size() * 4, hipMemcpyHostToDevice),
                   "upload");
}

// mantissa bytes of a block: n + 2 int32, rounded up to the 16-byte
// granularity of the zero fill
size_t vec_bytes(int n) { return ((size_t)(n + 2) * 4 + 15) & ~(size_t)15; }

int new_vec(fe_hierarchy* h, int n, int w, FeVec* v, hipStream_t s) {
  int rc;
  v->n = n;
  v->w = w;
  if ((rc = alloc(h, vec_bytes(n), (void**)&v->mant))) return rc;
  if ((rc = alloc(h, BFP_META_SLOTS * 8, (void**)&v->meta))) return rc;
  return hip_check(launch_init(v->mant, vec_bytes(n), v->meta, 1 - w, s), "init");
}

int bits_of(unsigned __int128 v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// z = Q_w_out(alpha M x + beta y) by qcomp; M null: the identity
int op(fe_hierarchy* h, const DevBand* M, const FeVec& x, const bfp_scalar& alpha, const FeVec* y,
       const bfp_scalar& beta, FeVec& z, int w_out, hipStream_t s) {
  if (w_out < 1 || w_out > 32) return fail(BFP_EWIDTH, "output width %d outside 1..32", w_out);
  const int64_t rowabs = M ? M->rowabs : 1;
  const unsigned __int128 am = (unsigned __int128)(alpha.m < 0 ? -alpha.m : alpha.m);
  const int abits = bits_of(am * (unsigned __int128)rowabs << (x.w - 1));
  const int bbits = y ? bits_of((unsigned __int128)(beta.m < 0 ? -beta.m : beta.m) << (y->w - 1)) : 0;
  if (abits > 61 || bbits > 61)
    return fail(BFP_EWIDTH, "an exact term may exceed the 61-bit budget (widths too large)");
  BandLaunch L;
  std::memset(&L, 0, sizeof L);
  L.op.w_out = w_out;
  L.op.has_y = y != nullptr;
  L.op.e_A = M ? M->e : 0;
  L.op.alpha_m = alpha.m;
  L.op.alpha_e = alpha.exp;
  L.op.beta_m = y ? beta.m : 0;
  L.op.beta_e = y ? beta.exp : 0;
  L.op.x_meta = x.meta;
  L.op.y_meta = y ? y->meta : x.meta;
  L.op.z_meta = z.meta;
  L.op.lo = -((int64_t)1 << (w_out - 1));
  L.op.hi = ((int64_t)1 << (w_out - 1)) - 1;
  L.op.abits = abits;
  L.op.bbits = bbits;
  L.x = x.mant;
  L.y = y ? y->mant : nullptr;
  L.z = z.mant;
  L.nout = z.n;
  L.col0 = M ? M->col0 : nullptr;
  L.taps = M ? M->taps : nullptr;
  L.band = M ? M->band : 0;
  int rc;
  if (h->rec) {   // recording the program: no launch
    if (z.n > kBandOneMax) h->rec_ok = false;
    BandStep st;
    std::memset(&st, 0, sizeof st);
    st.L = L;
    st.u = (int)((z.n + kBlock - 1) / kBlock);
    h->rec->push_back(st);
    z.w = w_out;
    h->prog_bytes += 4.0 * (double)x.n + (y ? 4.0 * y->n : 0) + 4.0 * z.n;
    return BFP_OK;
  }
  if (z.n <= fe_one_launch() && z.n <= kBandOneMax) {   // both passes in one launch
    if ((rc = hip_check(launch_band_qcomp1(L, s), "fe op (qcomp)"))) return rc;
    h->launches += 1;
  } else {
    L.op.mode = kModeQ1;
    if ((rc = hip_check(launch_band(L, s), "fe op (qcomp pass 1)"))) return rc;
    L.op.mode = kModeQ2;
    if ((rc = hip_check(launch_band(L, s), "fe op (qcomp pass 2)"))) return rc;
    h->launches += 2;
  }
  z.w = w_out;
  h->bytes += 4.0 * (M ? (double)x.n : (double)x.n) + (y ? 4.0 * y->n : 0) + 4.0 * z.n;
  return BFP_OK;
}

const bfp_scalar kOne{1, 0, 2}, kMinusOne{-1, 0, 1};

int vcycle(fe_hierarchy* h, int l, FeVec& rin, hipStream_t s) {
  const fe_params& p = h->prm;
  const int wi = p.w_inner[l];
  int rc;
  // relaxation y = c2 A r + c1 r
  if ((rc = op(h, &h->A_inner[l], rin, h->c2, &rin, h->c1, h->y[l], wi, s))) return rc;
  if (l > 1) {
    if ((rc = op(h, &h->A_inner[l], h->y[l], kOne, &rin, kMinusOne, h->rv[l], wi, s))) return rc;
    if ((rc = op(h, &h->R_inner[l], h->rv[l], kOne, nullptr, kOne, h->vin[l - 1], wi, s))) return rc;
    if ((rc = vcycle(h, l - 1, h->vin[l - 1], s))) return rc;
    if ((rc = op(h, &h->P_inner[l], h->y[l - 1], kMinusOne, &h->y[l], kOne, h->y[l], wi, s)))
      return rc;
  }
  return BFP_OK;
}

int ir_iteration(fe_hierarchy* h, int l, hipStream_t s) {
  const fe_params& p = h->prm;
  int rc;
  if ((rc = op(h, &h->A_check[l], h->x[l], kOne, &h->b[l], kMinusOne, h->r[l], p.w_inner[l], s)))
    return rc;
  if ((rc = vcycle(h, l, h->r[l], s))) return rc;
  return op(h, nullptr, h->x[l], kOne, &h->y[l], kMinusOne, h->x[l], p.w_work[l], s);
}

// FMG: x_1 = 0, then on each level l the prolongation of x_{l-1} (l > 1)
// and N IR iterations; launches the ops, or appends them to the program
// being recorded.
int fmg_sequence(fe_hierarchy* h, hipStream_t s) {
  const fe_params& p = h->prm;
  int rc;
  // x_1 = 0
  if (h->rec) {
    BandStep st;
    std::memset(&st, 0, sizeof st);
    st.init_mant = h->x[1].mant;
    st.init_words = (int64_t)(vec_bytes(h->n[1]) / 4);
    st.init_meta = h->x[1].meta;
    st.init_exp = 1 - p.w_work[1];
    h->rec->push_back(st);
  } else if ((rc = hip_check(launch_init(h->x[1].mant, vec_bytes(h->n[1]), h->x[1].meta,
                                         1 - p.w_work[1], s), "fe_fmg"))) {
    return rc;
  }
  h->x[1].w = p.w_work[1];
  for (int l = 1; l <= p.L; ++l) {
    if (l > 1 && (rc = op(h, &h->P_work[l], h->x[l - 1], kOne, nullptr, kOne, h->x[l], p.w_work[l], s)))
      return rc;
    for (int i = 0; i < p.N; ++i)
      if ((rc = ir_iteration(h, l, s))) return rc;
  }
  return BFP_OK;
}

// Record the whole FMG as one program (no launch); the hierarchy keeps
// running op by op when an op does not fit one workgroup or recording fails.
int record_program(fe_hierarchy* h, hipStream_t s) {
  std::vector<BandStep> steps;
  h->rec = &steps;
  h->rec_ok = true;
  h->prog_bytes = 0;
  const int rc = fmg_sequence(h, s);
  h->rec = nullptr;
  if (rc || !h->rec_ok || steps.empty() || steps.size() > (size_t)INT32_MAX) return BFP_OK;
  BandStep* d = nullptr;
  int e = alloc(h, steps.size() * sizeof(BandStep), (void**)&d);
  if (e) return e;
  if ((e = hip_check(hipMemcpy(d, steps.data(), steps.size() * sizeof(BandStep), hipMemcpyHostToDevice),
                     "upload")))
    return e;
  h->prog = d;
  h->prog_steps = (int)steps.size();
  return BFP_OK;
}

int quantize_scalar(const Q& q, int w, bfp_scalar* out) {
  if (q.n == 0) {
    *out = bfp_scalar{0, 1 - w, w};
    return BFP_OK;
  }
  const int e = nu_q(q) - w;
  out->m = (int64_t)floor_div_pow2(q, e);
  out->exp = e;
  out->w = w;
  return BFP_OK;
}

}  // namespace

extern "C" {

int fe_hierarchy_create(const fe_params* prm, const fe_rational_band* K, const fe_rational_band* P,
                        const double* const* F, void* stream, fe_hierarchy** out) {
  if (!prm || !K || !F || !out) return fail(BFP_EINVAL, "NULL argument");
  const int L = prm->L, m = prm->m;
  if (m != 1 && m != 2) return fail(BFP_EINVAL, "m must be 1 (Poisson) or 2 (biharmonic)");
  if (L < 1 || L > MG_MAX_LEVELS) return fail(BFP_ESHAPE, "L must be in 1..%d", MG_MAX_LEVELS);
  if (L > 1 && !P) return fail(BFP_EINVAL, "P is NULL");
  if (prm->N < 1) return fail(BFP_EINVAL, "N must be >= 1");
  if (prm->eta_num <= 0 || prm->eta_den <= prm->eta_num)
    return fail(BFP_EINVAL, "need 0 < eta < 1");
  for (int j = 1; j <= L; ++j)
    if (prm->w_check[j] < 1 || prm->w_check[j] > 32 || prm->w_work[j] < 1 || prm->w_work[j] > 32 ||
        prm->w_inner[j] < 1 || prm->w_inner[j] > 32)
      return fail(BFP_EWIDTH, "level %d: widths must be in 1..32", j);
  hipStream_t s = (hipStream_t)stream;
  fe_hierarchy* h = new (std::nothrow) fe_hierarchy();
  if (!h) return fail(BFP_ENOMEM, "host allocation failed");
  h->prm = *prm;
  int rc = BFP_OK;
  std::vector<RBand> A(L + 1), R(L + 1), Pr(L + 1);
  std::vector<std::vector<Q>> dg(L + 1);
  auto bad = [&](const char* what) {
    fe_hierarchy_destroy(h);
    return fail(BFP_EWIDTH, "%s does not fit 128-bit exact arithmetic", what);
  };
  for (int j = 1; j <= L && !rc; ++j) {
    RBand Kj;
    if ((rc = band_from_input(&K[j - 1], &Kj))) break;
    if (Kj.nrows != Kj.ncols) { rc = fail(BFP_ESHAPE, "K_%d is not square", j); break; }
    h->n[j] = Kj.nrows;
    dg[j].resize(Kj.nrows);
    for (int i = 0; i < Kj.nrows; ++i) {
      const int t = i - Kj.col0[i];
      if (t < 0 || t >= (int)Kj.v[i].size() || Kj.v[i][t].n <= 0) {
        rc = fail(BFP_EINVAL, "K_%d: diagonal entry %d missing or not positive", j, i);
        break;
      }
      dg[j][i] = Kj.v[i][t];
    }
    if (rc) break;
    A[j] = Kj;
    for (int i = 0; i < Kj.nrows; ++i)
      for (Q& q : A[j].v[i])
        if (!divq(q, dg[j][i], &q)) return bad("A");
  }
  for (int j = 2; j <= L && !rc; ++j) {
    if ((rc = band_from_input(&P[j - 1], &Pr[j]))) break;
    if (Pr[j].nrows != h->n[j] || Pr[j].ncols != h->n[j - 1]) {
      rc = fail(BFP_ESHAPE, "P_%d must map %d unknowns to %d", j, h->n[j - 1], h->n[j]);
      break;
    }
    // R = 2^(2m-1) Dc^-1 P^T Df
    std::vector<std::vector<std::pair<int, Q>>> cols(Pr[j].ncols);
    for (int k = 0; k < Pr[j].nrows; ++k)
      for (size_t t = 0; t < Pr[j].v[k].size(); ++t)
        if (Pr[j].v[k][t].n != 0) cols[Pr[j].col0[k] + t].push_back({k, Pr[j].v[k][t]});
    R[j].nrows = Pr[j].ncols;
    R[j].ncols = Pr[j].nrows;
    R[j].col0.resize(R[j].nrows);
    R[j].v.resize(R[j].nrows);
    for (int l = 0; l < R[j].nrows; ++l) {
      if (cols[l].empty()) { rc = fail(BFP_EINVAL, "P_%d has an empty column", j); break; }
      const int lo = cols[l].front().first, hi = cols[l].back().first;
      R[j].col0[l] = lo;
      R[j].v[l].assign(hi - lo + 1, Q{0, 1});
      for (auto& kv : cols[l]) {
        Q q;
        if (!mul(kv.second, dg[j][kv.first], &q) || !divq(q, dg[j - 1][l], &q) ||
            !mul_pow2(q, 2 * m - 1, &q))
          return bad("R");
        R[j].v[l][kv.first - lo] = q;
      }
    }
  }
  if (rc) {
    fe_hierarchy_destroy(h);
    return rc;
  }
  // Chebyshev coefficients from the Gershgorin bound on level min(5, L)
  {
    const int je = std::min(5, L);
    Q rho{0, 1};
    for (const auto& row : A[je].v) {
      Q s{0, 1};
      for (const Q& q : row)
        if (!add(s, Q{iabs(q.n), q.d}, &s)) return bad("rho");
      Q diff;
      if (!add(s, Q{-rho.n, rho.d}, &diff)) return bad("rho");
      if (diff.n > 0) rho = s;
    }
    const Q eta{prm->eta_num, prm->eta_den};
    Q one{1, 1}, two{2, 1}, half{1, 2}, alpha, c, beta, t;
    // alpha = (1 + eta) rho / 2, c = (1 - eta) rho / 2, beta = alpha - c^2 / (2 alpha)
    if (!add(one, eta, &t) || !mul(t, rho, &t) || !mul(t, half, &alpha)) return bad("c1");
    if (!add(one, Q{-eta.n, eta.d}, &t) || !mul(t, rho, &t) || !mul(t, half, &c)) return bad("c1");
    Q c2sq, twoa;
    if (!mul(c, c, &c2sq) || !mul(two, alpha, &twoa) || !divq(c2sq, twoa, &t) ||
        !add(alpha, Q{-t.n, t.d}, &beta))
      return bad("c1");
    Q c1q, c2q, ab;
    if (!divq(two, beta, &c1q) || !mul(alpha, beta, &ab) || !divq(Q{-1, 1}, ab, &c2q)) return bad("c2");
    quantize_scalar(c1q, 16, &h->c1);
    quantize_scalar(c2q, 16, &h->c2);
  }
  // operators per call site, blocks, right-hand sides
  for (int j = 1; j <= L && !rc; ++j) {
    rc = quantize_upload(h, A[j], prm->w_check[j], &h->A_check[j]);
    if (!rc) rc = quantize_upload(h, A[j], prm->w_inner[j], &h->A_inner[j]);
    if (!rc && j > 1) rc = quantize_upload(h, R[j], prm->w_inner[j], &h->R_inner[j]);
    if (!rc && j > 1) rc = quantize_upload(h, Pr[j], prm->w_inner[j], &h->P_inner[j]);
    if (!rc && j > 1) rc = quantize_upload(h, Pr[j], prm->w_work[j], &h->P_work[j]);
    const int n = h->n[j];
    if (!rc) rc = new_vec(h, n, prm->w_work[j], &h->x[j], s);
    if (!rc) rc = new_vec(h, n, prm->w_check[j], &h->b[j], s);
    if (!rc) rc = new_vec(h, n, prm->w_inner[j], &h->r[j], s);
    if (!rc) rc = new_vec(h, n, prm->w_inner[j], &h->y[j], s);
    if (!rc) rc = new_vec(h, n, prm->w_inner[j], &h->rv[j], s);
    if (!rc) rc = new_vec(h, n, j < L ? prm->w_inner[j + 1] : prm->w_inner[j], &h->vin[j], s);
    if (rc) break;
    // b_j = Q_w(2^(-2mj) F_hat / diag)
    if (!F[j - 1]) { rc = fail(BFP_EINVAL, "F_%d is NULL", j); break; }
    std::vector<Q> bq(n);
    int numax = INT32_MIN;
    for (int i = 0; i < n; ++i) {
      Q q;
      if (!std::isfinite(F[j - 1][i])) { rc = fail(BFP_ENONFINITE, "F_%d has a non-finite entry", j); break; }
      if (!from_double(F[j - 1][i], &q) || !mul_pow2(q, -2 * m * j, &q) || !divq(q, dg[j][i], &q))
        return bad("b");
      bq[i] = q;
      if (q.n != 0) numax = std::max(numax, nu_q(q));
    }
    if (rc) break;
    const int w = prm->w_check[j];
    const int64_t e = numax == INT32_MIN ? 1 - w : (int64_t)numax - w;
    std::vector<int32_t> mant(n + 2, 0);
    int64_t mx = 0, mn = 0;
    for (int i = 0; i < n; ++i) {
      const int64_t v = (int64_t)floor_div_pow2(bq[i], (int)e);
      mant[i + 1] = (int32_t)v;
      mx = std::max(mx, v);
      mn = std::min(mn, v);
    }
    const int64_t meta3[3] = {e, mx, mn};
    rc = hip_check(hipStreamSynchronize(s), "init");
    if (!rc) rc = hip_check(hipMemcpy(h->b[j].mant, mant.data(), (n + 2) * 4, hipMemcpyHostToDevice), "upload");
    if (!rc) rc = hip_check(hipMemcpy(h->b[j].meta, meta3, sizeof meta3, hipMemcpyHostToDevice), "upload");
  }
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "fe_hierarchy_create");
  if (!rc) rc = record_program(h, s);
  if (rc) {
    fe_hierarchy_destroy(h);
    return rc;
  }
  *out = h;
  return BFP_OK;
}

int fe_fmg(fe_hierarchy* h, void* stream) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  hipStream_t s = (hipStream_t)stream;
  if (h->prog && fe_program()) {   // the recorded program: one launch
    int rc = hip_check(launch_band_prog(h->prog, h->prog_steps, s), "fe_fmg (program)");
    if (rc) return rc;
    h->launches += 1;
    h->bytes += h->prog_bytes;
    return BFP_OK;
  }
  return fmg_sequence(h, s);
}

int fe_get(fe_hierarchy* h, int level, int which, int32_t* mant_host, int64_t* exp_out, int* n_out) {
  if (!h || level < 1 || level > h->prm.L || !exp_out || !n_out)
    return fail(BFP_EINVAL, "bad argument");
  const FeVec* v = which == 0 ? &h->x[level] : which == 1 ? &h->b[level] : which == 2 ? &h->r[level]
                                                                                    : nullptr;
  if (!v) return fail(BFP_EINVAL, "unknown block %d", which);
  int rc = hip_check(hipDeviceSynchronize(), "fe_get");
  if (rc) return rc;
  *n_out = v->n;
  int64_t e = 0;
  if ((rc = hip_check(hipMemcpy(&e, v->meta, 8, hipMemcpyDeviceToHost), "fe_get"))) return rc;
  *exp_out = e;
  if (mant_host)
    rc = hip_check(hipMemcpy(mant_host, v->mant, (size_t)(v->n + 2) * 4, hipMemcpyDeviceToHost), "fe_get");
  return rc;
}

int fe_coefficients(const fe_hierarchy* h, bfp_scalar* c1, bfp_scalar* c2) {
  if (!h || !c1 || !c2) return fail(BFP_EINVAL, "NULL argument");
  *c1 = h->c1;
  *c2 = h->c2;
  return BFP_OK;
}

int fe_counters(const fe_hierarchy* h, double* bytes, int64_t* launches) {
  if (!h) return fail(BFP_EINVAL, "NULL hierarchy");
  if (bytes) *bytes = h->bytes;
  if (launches) *launches = h->launches;
  return BFP_OK;
}

int fe_hierarchy_destroy(fe_hierarchy* h) {
  if (!h) return BFP_OK;
  for (void* p : h->allocs) (void)hipFree(p);
  delete h;
  return BFP_OK;
}

}  // extern "C"
