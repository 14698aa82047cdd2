// A priori estimation of the BFP precisions (Section 6.2, Algorithm
// bfp-prec-est) and of the Chebyshev parameter eta (Section 5).
//
// conv-rate-v-cycle: the error propagation matrix E of one BFP IR-V
// iteration on the estimation level (b = 0, so the new iterate is the
// propagated error) is built column by column on the device, by running the
// library's IR iteration on the canonical basis vectors; its rate is the
// energy norm rho_v = ||E||_A, the square root of the largest generalized
// eigenvalue of E^T A E x = lambda A x.
//
// The energy norm is computed on the host without a dense eigensolver: the
// scaled 5- and 7-point operators are diagonalized by the orthonormal sine
// transform S (A = S Lambda S), so ||E||_A = ||Lambda^1/2 (S E S)
// Lambda^-1/2||_2, whose square is the largest eigenvalue of G^T G, found by
// Lanczos with full reorthogonalization and Sturm bisection on the
// tridiagonal matrix.
//
// bfp-prec-est: the width rules check_j(q) = j (m + k) + q and
// inner_j(q) = j m + q; the reference rate at q_max; the smallest q in
// 1..q_max (binary search) whose rate stays below rho_thresh times the
// reference, first for the check width with the inner width at q_max, then
// for the inner width with that check width. Widths are capped at the
// 32-bit mantissa storage; the check width is kept at least the working
// width and the inner width at most the working width (the order of the
// three precisions); the working widths are the caller's.
//
// eta: the percentage i in lo..hi (i / 100 = the part of the spectrum the
// Chebyshev relaxation targets) whose V-cycle rate rho_v is smallest, every
// i evaluated (ties to the smallest i).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"
#include "kernels.hpp"

using namespace bfpk;

namespace {

// ------------------------------------------------------ energy norm ---

// v <- S v along every axis of an n^ndim block (S the orthonormal DST-I,
// symmetric and its own inverse); `line` is scratch of n doubles
void sine_transform(double* v, int ndim, int n, const std::vector<double>& S, double* line) {
  const int64_t N = ndim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
  for (int ax = 0; ax < ndim; ++ax) {
    const int64_t stride = ax == 0 ? 1 : (ax == 1 ? n : (int64_t)n * n);
    for (int64_t base = 0; base < N; ++base) {
      // base enumerates the lines along axis ax: its coordinate on that axis is 0
      if ((base / stride) % n != 0) continue;
      for (int a = 0; a < n; ++a) {
        double acc = 0;
        for (int b = 0; b < n; ++b) acc += S[(size_t)a * n + b] * v[base + b * stride];
        line[a] = acc;
      }
      for (int a = 0; a < n; ++a) v[base + a * stride] = line[a];
    }
  }
}

// largest eigenvalue of the symmetric tridiagonal matrix (a, b) by Sturm
// bisection: count(x) = number of eigenvalues below x
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int k = (int)a.size();
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::fmin(lo, a[i] - r);
    hi = std::fmax(hi, a[i] + r);
  }
  auto below = [&](double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = a[i] - x - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-16 * std::fmax(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) == k) hi = mid;
    else lo = mid;
  }
  return hi;
}

}  // namespace

extern "C" int bfp_energy_norm(const double* E, int ndim, int j, double* rho) {
  if (!E || !rho) return fail(BFP_EINVAL, "NULL argument");
  if ((ndim != 2 && ndim != 3) || j < 1 || j > (ndim == 2 ? 7 : 5))
    return fail(BFP_ESHAPE, "energy norm: ndim 2 with level 1..7 or ndim 3 with level 1..5");
  const int n = (1 << j) - 1;
  const int64_t N = ndim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
  std::vector<double> S((size_t)n * n), lam(N), line(n);
  const double sc = std::sqrt(2.0 / (n + 1));
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) S[(size_t)a * n + b] = sc * std::sin(M_PI * (a + 1) * (b + 1) / (n + 1));
  // eigenvalues of the operator scaled to unit diagonal, 1 - mean_k cos(pi k_k h)
  for (int64_t i = 0; i < N; ++i) {
    double c = 0;
    int64_t r = i;
    for (int ax = 0; ax < ndim; ++ax) {
      c += std::cos(M_PI * (double)(r % n + 1) / (n + 1));
      r /= n;
    }
    lam[i] = 1.0 - c / ndim;
  }
  // G = Lambda^1/2 S E S Lambda^-1/2, G[col k][row i] (columns contiguous)
  std::vector<double> G((size_t)(N * N));
  std::memcpy(G.data(), E, sizeof(double) * (size_t)(N * N));
  for (int64_t k = 0; k < N; ++k) sine_transform(&G[k * N], ndim, n, S, line.data());
  std::vector<double> row(N);
  for (int64_t i = 0; i < N; ++i) {   // right factor: rows of S E, transformed
    for (int64_t k = 0; k < N; ++k) row[k] = G[k * N + i];
    sine_transform(row.data(), ndim, n, S, line.data());
    for (int64_t k = 0; k < N; ++k) G[k * N + i] = row[k];
  }
  for (int64_t k = 0; k < N; ++k)
    for (int64_t i = 0; i < N; ++i) G[k * N + i] *= std::sqrt(lam[i] / lam[k]);
  // Lanczos on G^T G from a fixed start vector, fully reorthogonalized
  const int kmax = (int)std::min<int64_t>(N, 400);
  std::vector<double> Q((size_t)kmax * N), u(N), w(N), al, be;
  uint64_t st = 0x9e3779b97f4a7c15ull;
  double nrm = 0;
  for (int64_t i = 0; i < N; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    Q[i] = 1.0 + (double)(st >> 11) * (1.0 / 9007199254740992.0);
    nrm += Q[i] * Q[i];
  }
  for (int64_t i = 0; i < N; ++i) Q[i] /= std::sqrt(nrm);
  double theta = 0, prev = -1;
  int stable = 0;
  for (int k = 0; k < kmax; ++k) {
    const double* q = &Q[(size_t)k * N];
    for (int64_t i = 0; i < N; ++i) u[i] = 0;
    for (int64_t c = 0; c < N; ++c) {            // u = G q
      const double qc = q[c];
      const double* g = &G[c * N];
      for (int64_t i = 0; i < N; ++i) u[i] += g[i] * qc;
    }
    for (int64_t c = 0; c < N; ++c) {            // w = G^T u
      const double* g = &G[c * N];
      double acc = 0;
      for (int64_t i = 0; i < N; ++i) acc += g[i] * u[i];
      w[c] = acc;
    }
    double a = 0;
    for (int64_t i = 0; i < N; ++i) a += q[i] * w[i];
    al.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (int m = 0; m <= k; ++m) {
        const double* qm = &Q[(size_t)m * N];
        double d = 0;
        for (int64_t i = 0; i < N; ++i) d += qm[i] * w[i];
        for (int64_t i = 0; i < N; ++i) w[i] -= d * qm[i];
      }
    double bn = 0;
    for (int64_t i = 0; i < N; ++i) bn += w[i] * w[i];
    bn = std::sqrt(bn);
    theta = tridiag_max_eig(al, be);
    if (k + 1 == kmax || bn <= 1e-14 * std::fmax(theta, 1e-300)) break;
    stable = std::fabs(theta - prev) <= 1e-14 * theta ? stable + 1 : 0;
    if (stable >= 3 && k >= 8) break;
    prev = theta;
    be.push_back(bn);
    double* qn = &Q[(size_t)(k + 1) * N];
    for (int64_t i = 0; i < N; ++i) qn[i] = w[i] / bn;
  }
  *rho = std::sqrt(std::fmax(theta, 0.0));
  return BFP_OK;
}

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t interior_count(int ndim, int j) {
  const int64_t n = ((int64_t)1 << j) - 1;
  return ndim == 2 ? n * n : n * n * n;
}
int64_t padded_count(int ndim, int j) {
  const int64_t s = ((int64_t)1 << j) + 1;
  return ndim == 2 ? s * s : s * s * s;
}

int check_est(const mg_params* p) {
  if (!p) return fail(BFP_EINVAL, "params are NULL");
  if ((p->ndim == 2 && p->L > 7) || (p->ndim == 3 && p->L > 5))
    return fail(BFP_ESHAPE, "estimation level must be at most 7 (2D) or 5 (3D)");
  return params_ok(p);
}

}  // namespace

extern "C" {

size_t mg_conv_rate_bytes(const mg_params* prm) {
  if (check_est(prm)) return 0;
  size_t hb = 0;
  if (hierarchy_bytes_ex(prm, exec_max_points(), &hb)) return 0;
  const int64_t N = interior_count(prm->ndim, prm->L);
  return align256(hb) + align256(sizeof(double) * (size_t)(N * padded_count(prm->ndim, prm->L)));
}

int mg_error_propagation(const mg_params* prm, void* arena_dev, size_t bytes, void* stream,
                         double* E_host) {
  int rc = check_est(prm);
  if (rc) return rc;
  if (!arena_dev || !E_host) return fail(BFP_EINVAL, "NULL argument");
  const size_t need = mg_conv_rate_bytes(prm);
  if (bytes < need) return fail(BFP_ENOMEM, "arena holds %zu bytes, the estimation needs %zu", bytes, need);
  size_t hb = 0;
  if ((rc = hierarchy_bytes_ex(prm, exec_max_points(), &hb))) return rc;
  hipStream_t s = (hipStream_t)stream;
  mg_hierarchy* h = nullptr;
  if ((rc = hierarchy_create_ex(prm, arena_dev, hb, stream, exec_max_points(), &h))) return rc;
  const int ndim = prm->ndim, j = prm->L;
  const int64_t n = ((int64_t)1 << j) - 1, side = n + 2;
  const int64_t N = interior_count(ndim, j), P = padded_count(ndim, j);
  double* cols = reinterpret_cast<double*>(static_cast<char*>(arena_dev) + align256(hb));
  bfp_vec x;
  if ((rc = mg_get_vec(h, j, 0, &x))) { mg_hierarchy_destroy(h); return rc; }
  // b = 0 on every level: the hierarchy starts zeroed
  for (int64_t k = 0; k < N && !rc; ++k) {
    const int64_t ix = k % n + 1, iy = (k / n) % n + 1, iz = ndim == 3 ? k / (n * n) + 1 : 0;
    const int64_t pos = (ndim == 3 ? iz * side + iy : iy) * x.pitch + ix;
    if ((rc = bfp_vec_init(&x, stream))) break;
    if ((rc = hip_check(launch_unit(x.mant, x.storage_bits, pos, x.meta, x.w, s), "unit vector"))) break;
    if ((rc = mg_ir(h, j, 1, stream))) break;
    rc = bfp_vec_to_f64(&x, cols + k * P, stream);
  }
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "estimation columns");
  std::vector<double> host;
  if (!rc) {
    try { host.resize((size_t)(N * P)); } catch (...) { rc = fail(BFP_ENOMEM, "host allocation failed"); }
  }
  if (!rc) rc = hip_check(hipMemcpy(host.data(), cols, sizeof(double) * (size_t)(N * P),
                                    hipMemcpyDeviceToHost), "estimation columns");
  if (!rc) {
    for (int64_t k = 0; k < N; ++k)
      for (int64_t i = 0; i < N; ++i) {
        const int64_t ix = i % n + 1, iy = (i / n) % n + 1, iz = ndim == 3 ? i / (n * n) + 1 : 0;
        E_host[k * N + i] = host[(size_t)(k * P + (ndim == 3 ? (iz * side + iy) * side : iy * side) + ix)];
      }
  }
  mg_hierarchy_destroy(h);
  return rc;
}

int mg_conv_rate(const mg_params* prm, void* arena_dev, size_t bytes, void* stream, double* rho) {
  int rc = check_est(prm);
  if (rc) return rc;
  if (!rho) return fail(BFP_EINVAL, "NULL argument");
  const int64_t N = interior_count(prm->ndim, prm->L);
  std::vector<double> E;
  try { E.resize((size_t)(N * N)); } catch (...) { return fail(BFP_ENOMEM, "host allocation failed"); }
  if ((rc = mg_error_propagation(prm, arena_dev, bytes, stream, E.data()))) return rc;
  return bfp_energy_norm(E.data(), prm->ndim, prm->L, rho);
}

int mg_params_apply_estimate(mg_params* p, int q_check, int q_inner, int m, int k) {
  if (!p) return fail(BFP_EINVAL, "params are NULL");
  if (m < 1 || k < 1 || q_check < 1 || q_inner < 1)
    return fail(BFP_EINVAL, "need m, k, q_check, q_inner >= 1");
  for (int j = 1; j <= p->L; ++j) {
    const int work = p->w_work[j];
    int check = j * (m + k) + q_check;
    check = check > 32 ? 32 : check;
    p->w_check[j] = check < work ? work : check;
    const int inner = j * m + q_inner;
    p->w_inner[j] = inner > work ? work : inner;
  }
  return params_ok(p);
}

int mg_prec_est(const mg_params* base, int q_max, double rho_thresh, int m, int k,
                void* arena_dev, size_t bytes, void* stream, mg_prec_est_result* out) {
  int rc = check_est(base);
  if (rc) return rc;
  if (!out) return fail(BFP_EINVAL, "NULL argument");
  if (q_max < 1 || !(rho_thresh > 1.0)) return fail(BFP_EINVAL, "need q_max >= 1 and rho_thresh > 1");
  // rates of the width schedules met so far (the caps make many q equal)
  std::map<std::vector<int>, double> seen;
  auto rate = [&](int qc, int qi, double* r) {
    mg_params p = *base;
    int e = mg_params_apply_estimate(&p, qc, qi, m, k);
    if (e) return e;
    std::vector<int> key;
    for (int j = 1; j <= p.L; ++j) { key.push_back(p.w_check[j]); key.push_back(p.w_inner[j]); }
    auto it = seen.find(key);
    if (it != seen.end()) { *r = it->second; return (int)BFP_OK; }
    if ((e = mg_conv_rate(&p, arena_dev, bytes, stream, r))) return e;
    seen[key] = *r;
    return (int)BFP_OK;
  };
  // smallest q in 1..q_max with ok(q); ok(q_max) holds by construction
  auto smallest = [&](auto ok, int* q) {
    int lo = 1, hi = q_max;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      bool yes = false;
      int e = ok(mid, &yes);
      if (e) return e;
      if (yes) hi = mid;
      else lo = mid + 1;
    }
    *q = lo;
    return (int)BFP_OK;
  };
  double ref = 0;
  if ((rc = rate(q_max, q_max, &ref))) return rc;
  int qc = q_max, qi = q_max;
  rc = smallest([&](int q, bool* yes) {
    double r = 0;
    int e = rate(q, q_max, &r);
    *yes = r < rho_thresh * ref;
    return e;
  }, &qc);
  if (rc) return rc;
  rc = smallest([&](int q, bool* yes) {
    double r = 0;
    int e = rate(qc, q, &r);
    *yes = r < rho_thresh * ref;
    return e;
  }, &qi);
  if (rc) return rc;
  double fin = 0;
  if ((rc = rate(qc, qi, &fin))) return rc;
  out->q_check = qc;
  out->q_inner = qi;
  out->rho_ref = ref;
  out->rho = fin;
  out->rates = (int)seen.size();
  return BFP_OK;
}

int mg_eta_scan(const mg_params* base, int lo, int hi, void* arena_dev, size_t bytes,
                void* stream, int* eta_percent, double* rho, double* rates) {
  int rc = check_est(base);
  if (rc) return rc;
  if (!eta_percent || !rho) return fail(BFP_EINVAL, "NULL argument");
  if (lo < 1 || hi > 99 || lo > hi) return fail(BFP_EINVAL, "need 1 <= lo <= hi <= 99");
  int best = -1;
  double best_r = 0;
  for (int i = lo; i <= hi; ++i) {
    mg_params p = *base;
    if ((rc = set_smoother(&p, i))) return rc;
    double r = 0;
    if ((rc = mg_conv_rate(&p, arena_dev, bytes, stream, &r))) return rc;
    if (rates) rates[i - lo] = r;
    if (best < 0 || r < best_r) {
      best = i;
      best_r = r;
    }
  }
  *eta_percent = best;
  *rho = best_r;
  return BFP_OK;
}

}  // extern "C"
