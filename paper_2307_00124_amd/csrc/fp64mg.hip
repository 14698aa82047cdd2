// FP64 multigrid comparator: the same FMG / IR / V(nu1, nu2) schedule as the
// BFP solver (Appendix C with the readings of the BFP driver) on the same
// scaled operators (2D: A' = [1; -1/4], R' = P^T, bilinear P; 3D:
// A' = [3/4; -1/8], R' = P^T / 2, trilinear P) with the same Chebyshev
// coefficients, in IEEE double arithmetic: the floating-point reference of
// the "BFP vs FP64 multigrid" comparison. No quantization, no norms and no
// reductions: every operation is a plain streaming kernel, and the levels
// of at most kF64CoarsePts points run inside one single-workgroup launch
// (the V-cycle below them, or the coarse FMG levels), like the BFP solver's
// coarse-level executor.
//
// Layout: level j holds dense (n_j + 2)^ndim doubles with a zero Dirichlet
// ring, rows padded to 16 doubles (128 bytes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"

using namespace bfpk;

namespace {

constexpr int kF64Block = 256;
constexpr int kF64CoarseThreads = 512;
constexpr int64_t kF64CoarsePts = 4096;
constexpr int kF64MaxBlocks = 4096;

struct Lev64 {
  int64_t n, pitch;          // interior points per dimension, row pitch (doubles)
  double *x, *b, *r, *y, *s, *t, *rc;
};

// one operation's grid description
struct G64 {
  int64_t n, pitch;
};

__device__ __forceinline__ int64_t rows_of(int ND, int64_t n) { return ND == 3 ? n * n : n; }
__device__ __forceinline__ int64_t row_index(int ND, int64_t r, int64_t n) {
  // interior row number r (0-based) -> padded row index
  return ND == 3 ? (r / n + 1) * (n + 2) + (r % n + 1) : r + 1;
}

// z = alpha (A x) + beta y for the star operator (centre c0, faces co);
// y may be null or alias z (not x); points of interior row r, column c
template <int ND>
__device__ __forceinline__ double star_at(const double* x, int64_t rowp, int64_t pitch, int64_t side,
                                          int64_t c, double c0, double co) {
  const int64_t i = rowp * pitch + c;
  double s = x[i - 1] + x[i + 1] + x[i - pitch] + x[i + pitch];
  if (ND == 3) s += x[i - side * pitch] + x[i + side * pitch];
  return c0 * x[i] + co * s;
}

template <int ND>
__device__ __forceinline__ void op_gemv(int64_t t0, int64_t nt, const G64 g, const double* x,
                                        const double* y, double* z, double alpha, double beta,
                                        double c0, double co) {
  const int64_t n = g.n, side = n + 2, total = rows_of(ND, n) * n;
  for (int64_t k = t0; k < total; k += nt) {
    const int64_t r = k / n, c = k % n + 1;
    const int64_t rowp = row_index(ND, r, n);
    const int64_t i = rowp * g.pitch + c;
    double v = alpha * star_at<ND>(x, rowp, g.pitch, side, c, c0, co);
    if (y) v += beta * y[i];
    z[i] = v;
  }
}

template <int ND>
__device__ __forceinline__ void op_sub(int64_t t0, int64_t nt, const G64 g, const double* x,
                                       const double* y, double* z) {
  const int64_t n = g.n, total = rows_of(ND, n) * n;
  for (int64_t k = t0; k < total; k += nt) {
    const int64_t r = k / n, c = k % n + 1;
    const int64_t i = row_index(ND, r, n) * g.pitch + c;
    z[i] = x[i] - y[i];
  }
}

// 1D weights of the transfers: offset 0 -> 1, offset +-1 -> 1/2
__device__ __forceinline__ double w1(int o) { return o == 0 ? 1.0 : 0.5; }

// coarse rc[I] = s * sum_o w(o) f[2I + o], s = 1/4 (2D, R' = P^T with
// P = bilinear) or 1/2 (3D: R' = P^T / 2 with the product weights)
template <int ND>
__device__ __forceinline__ void op_restrict(int64_t t0, int64_t nt, const G64 gf, const G64 gc,
                                            const double* f, double* rc) {
  const int64_t nc = gc.n, total = rows_of(ND, nc) * nc;
  const int64_t sf = gf.n + 2, sc = nc + 2;
  const double scale = ND == 2 ? 1.0 : 0.5;
  for (int64_t k = t0; k < total; k += nt) {
    const int64_t r = k / nc, cx = k % nc + 1;
    const int64_t cz = ND == 3 ? r / nc + 1 : 0, cy = ND == 3 ? r % nc + 1 : r + 1;
    double acc = 0;
    for (int oz = (ND == 3 ? -1 : 0); oz <= (ND == 3 ? 1 : 0); ++oz)
      for (int oy = -1; oy <= 1; ++oy) {
        const int64_t frow = ND == 3 ? (2 * cz + oz) * sf + (2 * cy + oy) : 2 * cy + oy;
        const double* fr = f + frow * gf.pitch + 2 * cx;
        const double wyz = w1(oy) * (ND == 3 ? w1(oz) : 1.0);
        acc += wyz * (0.5 * fr[-1] + fr[0] + 0.5 * fr[1]);
      }
    rc[(ND == 3 ? cz * sc + cy : cy) * gc.pitch + cx] = scale * acc;
  }
}

// fine z[p] = alpha * (P d)[p] + beta * y[p] (y may be null or alias z)
template <int ND>
__device__ __forceinline__ void op_prolong(int64_t t0, int64_t nt, const G64 gc, const G64 gf,
                                           const double* d, const double* y, double* z,
                                           double alpha, double beta) {
  const int64_t nf = gf.n, total = rows_of(ND, nf) * nf;
  const int64_t sf = nf + 2, sc = gc.n + 2;
  for (int64_t k = t0; k < total; k += nt) {
    const int64_t r = k / nf, fx = k % nf + 1;
    const int64_t fz = ND == 3 ? r / nf + 1 : 0, fy = ND == 3 ? r % nf + 1 : r + 1;
    double acc = 0;
    // coarse J with |2J - p| <= 1: along each axis J = p/2 (even p) or (p -+ 1)/2
    const int nzs = ND == 3 ? ((fz & 1) ? 2 : 1) : 1, nys = (fy & 1) ? 2 : 1, nxs = (fx & 1) ? 2 : 1;
    for (int a = 0; a < nzs; ++a) {
      const int64_t jz = ND == 3 ? ((fz & 1) ? (fz - 1) / 2 + a : fz / 2) : 0;
      const double wz = ND == 3 ? ((fz & 1) ? 0.5 : 1.0) : 1.0;
      for (int b2 = 0; b2 < nys; ++b2) {
        const int64_t jy = (fy & 1) ? (fy - 1) / 2 + b2 : fy / 2;
        const double wy = (fy & 1) ? 0.5 : 1.0;
        const double* dr = d + (ND == 3 ? jz * sc + jy : jy) * gc.pitch;
        for (int c = 0; c < nxs; ++c) {
          const int64_t jx = (fx & 1) ? (fx - 1) / 2 + c : fx / 2;
          const double wx = (fx & 1) ? 0.5 : 1.0;
          acc += wz * wy * wx * dr[jx];
        }
      }
    }
    const int64_t i = (ND == 3 ? fz * sf + fy : fy) * gf.pitch + fx;
    double v = alpha * acc;
    if (y) v += beta * y[i];
    z[i] = v;
  }
}

// b = f * 2^k over the whole padded grid (ring of f ignored: written 0)
template <int ND>
__device__ __forceinline__ void op_scale(int64_t t0, int64_t nt, const G64 g, const double* f,
                                         double* b, double s) {
  const int64_t n = g.n, side = n + 2, total = rows_of(ND, n) * n;
  for (int64_t k = t0; k < total; k += nt) {
    const int64_t r = k / n, c = k % n + 1;
    const int64_t rowp = row_index(ND, r, n);
    b[rowp * g.pitch + c] = s * f[rowp * side + c];
  }
}

// zero the padded grid (ring and padding included)
__device__ __forceinline__ void op_zero(int64_t t0, int64_t nt, int64_t count, double* p) {
  for (int64_t k = t0; k < count; k += nt) p[k] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------- solver --

struct fp64_mg {
  int ndim, L, nu1, nu2, N, Lc;
  double c1, c2;         // relaxation y = c2 A' r + c1 r for the stored A'
  double c0, co;         // A' = [c0; co]
  Lev64 lv[MG_MAX_LEVELS + 1];
  Lev64* lv_dev;         // copy of lv for the coarse-level kernel
};

namespace {

template <int ND>
struct Ctx {
  const Lev64* lv;
  double c1, c2, c0, co;
  int nu1, nu2, N;
};

// The whole V(nu1, nu2) cycle from level l down, by one workgroup.
template <int ND>
__device__ void coarse_vcycle(const Ctx<ND>& C, int l, const double* rin) {
  const int64_t t0 = threadIdx.x, nt = blockDim.x;
  // descend: relaxation (and the added pre-sweeps), residual, restriction
  for (int k = l; k >= 1; --k) {
    const Lev64& v = C.lv[k];
    const G64 g{v.n, v.pitch};
    const double* r = k == l ? rin : v.rc;
    op_gemv<ND>(t0, nt, g, r, r, v.y, C.c2, C.c1, C.c0, C.co);
    __syncthreads();
    for (int s = 1; s < C.nu1; ++s) {
      op_gemv<ND>(t0, nt, g, v.y, r, v.s, 1.0, -1.0, C.c0, C.co);
      __syncthreads();
      op_gemv<ND>(t0, nt, g, v.s, v.s, v.t, C.c2, C.c1, C.c0, C.co);
      __syncthreads();
      op_sub<ND>(t0, nt, g, v.y, v.t, v.y);
      __syncthreads();
    }
    if (k > 1) {
      op_gemv<ND>(t0, nt, g, v.y, r, v.s, 1.0, -1.0, C.c0, C.co);
      __syncthreads();
      const Lev64& c = C.lv[k - 1];
      op_restrict<ND>(t0, nt, g, G64{c.n, c.pitch}, v.s, c.rc);
      __syncthreads();
    }
  }
  // ascend: correction and the post-sweeps
  for (int k = 1; k <= l; ++k) {
    const Lev64& v = C.lv[k];
    const G64 g{v.n, v.pitch};
    const double* r = k == l ? rin : v.rc;
    if (k > 1) {
      const Lev64& c = C.lv[k - 1];
      op_prolong<ND>(t0, nt, G64{c.n, c.pitch}, g, c.y, v.y, v.y, -1.0, 1.0);
      __syncthreads();
    }
    for (int s = 0; s < C.nu2; ++s) {
      op_gemv<ND>(t0, nt, g, v.y, r, v.s, 1.0, -1.0, C.c0, C.co);
      __syncthreads();
      op_gemv<ND>(t0, nt, g, v.s, v.s, v.t, C.c2, C.c1, C.c0, C.co);
      __syncthreads();
      op_sub<ND>(t0, nt, g, v.y, v.t, v.y);
      __syncthreads();
    }
  }
}

template <int ND>
__global__ __launch_bounds__(kF64CoarseThreads) void k64_coarse(const Lev64* lv, int l, int fmg_levels,
                                                               double c1, double c2, double c0,
                                                               double co, int nu1, int nu2, int N,
                                                               int from_rc) {
  const Ctx<ND> C{lv, c1, c2, c0, co, nu1, nu2, N};
  const int64_t t0 = threadIdx.x, nt = blockDim.x;
  if (fmg_levels > 0) {
    // FMG on levels 1..fmg_levels from x_1 = 0
    for (int k = 1; k <= fmg_levels; ++k) {
      const Lev64& v = lv[k];
      const G64 g{v.n, v.pitch};
      if (k == 1) {
        const int64_t cnt = (ND == 3 ? (v.n + 2) * (v.n + 2) : (v.n + 2)) * v.pitch;
        op_zero(t0, nt, cnt, v.x);
      } else {
        const Lev64& c = lv[k - 1];
        op_prolong<ND>(t0, nt, G64{c.n, c.pitch}, g, c.x, nullptr, v.x, 1.0, 0.0);
      }
      __syncthreads();
      for (int i = 0; i < N; ++i) {
        op_gemv<ND>(t0, nt, g, v.x, v.b, v.r, 1.0, -1.0, c0, co);
        __syncthreads();
        coarse_vcycle<ND>(C, k, v.r);
        op_sub<ND>(t0, nt, g, v.x, v.y, v.x);
        __syncthreads();
      }
    }
    return;
  }
  coarse_vcycle<ND>(C, l, from_rc ? lv[l].rc : lv[l].r);
}

template <int ND>
__global__ __launch_bounds__(kF64Block) void k64_gemv(const G64 g, const double* x, const double* y,
                                                     double* z, double alpha, double beta, double c0,
                                                     double co) {
  op_gemv<ND>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, g,
              x, y, z, alpha, beta, c0, co);
}
template <int ND>
__global__ __launch_bounds__(kF64Block) void k64_sub(const G64 g, const double* x, const double* y,
                                                    double* z) {
  op_sub<ND>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, g, x,
             y, z);
}
template <int ND>
__global__ __launch_bounds__(kF64Block) void k64_restrict(const G64 gf, const G64 gc, const double* f,
                                                         double* rc) {
  op_restrict<ND>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x,
                  gf, gc, f, rc);
}
template <int ND>
__global__ __launch_bounds__(kF64Block) void k64_prolong(const G64 gc, const G64 gf, const double* d,
                                                        const double* y, double* z, double alpha,
                                                        double beta) {
  op_prolong<ND>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x,
                 gc, gf, d, y, z, alpha, beta);
}
template <int ND>
__global__ __launch_bounds__(kF64Block) void k64_scale(const G64 g, const double* f, double* b,
                                                      double s) {
  op_scale<ND>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, g,
               f, b, s);
}

unsigned blocks_for(int ndim, int64_t n) {
  const int64_t pts = ndim == 3 ? n * n * n : n * n;
  const int64_t b = (pts + kF64Block - 1) / kF64Block;
  return (unsigned)(b < kF64MaxBlocks ? (b < 1 ? 1 : b) : kF64MaxBlocks);
}

int64_t pitch64(int64_t n) { return ((n + 2 + 15) / 16) * 16; }
int64_t grid_doubles(int ndim, int64_t n) {
  return (ndim == 3 ? (n + 2) * (n + 2) : (n + 2)) * pitch64(n);
}
size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t layout64(fp64_mg* h, int ndim, int L, char* base) {
  size_t off = 0;
  for (int j = 1; j <= L; ++j) {
    Lev64& v = h->lv[j];
    v.n = ((int64_t)1 << j) - 1;
    v.pitch = pitch64(v.n);
    const size_t b = al256(sizeof(double) * (size_t)grid_doubles(ndim, v.n));
    double** f[] = {&v.x, &v.b, &v.r, &v.y, &v.s, &v.t, &v.rc};
    for (double** p : f) {
      *p = base ? reinterpret_cast<double*>(base + off) : nullptr;
      off += b;
    }
  }
  h->lv_dev = base ? reinterpret_cast<Lev64*>(base + off) : nullptr;
  off = al256(off + sizeof(Lev64) * (MG_MAX_LEVELS + 1));
  return off;
}

template <int ND>
int vcycle64(fp64_mg* h, int l, const double* r, hipStream_t s) {
  Lev64& v = h->lv[l];
  const G64 g{v.n, v.pitch};
  const unsigned nb = blocks_for(ND, v.n);
  if (l <= h->Lc) {
    // the whole cycle from level l down in one launch (r is v.r or v.rc)
    hipLaunchKernelGGL(k64_coarse<ND>, dim3(1), dim3(kF64CoarseThreads), 0, s, h->lv_dev, l, 0,
                       h->c1, h->c2, h->c0, h->co, h->nu1, h->nu2, h->N, r == v.rc ? 1 : 0);
    return hip_check(hipGetLastError(), "fp64 coarse cycle");
  }
  hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, r, r, v.y, h->c2, h->c1, h->c0,
                     h->co);
  for (int k = 1; k < h->nu1; ++k) {
    hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.y, r, v.s, 1.0, -1.0, h->c0, h->co);
    hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.s, v.s, v.t, h->c2, h->c1, h->c0, h->co);
    hipLaunchKernelGGL(k64_sub<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.y, v.t, v.y);
  }
  Lev64& c = h->lv[l - 1];
  const G64 gc{c.n, c.pitch};
  hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.y, r, v.s, 1.0, -1.0, h->c0, h->co);
  hipLaunchKernelGGL(k64_restrict<ND>, dim3(blocks_for(ND, c.n)), dim3(kF64Block), 0, s, g, gc, v.s, c.rc);
  int rc = vcycle64<ND>(h, l - 1, c.rc, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k64_prolong<ND>, dim3(nb), dim3(kF64Block), 0, s, gc, g, c.y, v.y, v.y, -1.0, 1.0);
  for (int k = 0; k < h->nu2; ++k) {
    hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.y, r, v.s, 1.0, -1.0, h->c0, h->co);
    hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.s, v.s, v.t, h->c2, h->c1, h->c0, h->co);
    hipLaunchKernelGGL(k64_sub<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.y, v.t, v.y);
  }
  return hip_check(hipGetLastError(), "fp64 V-cycle");
}

template <int ND>
int fmg64(fp64_mg* h, const double* const* rhs, double* x_out, hipStream_t s) {
  // b_j = f_j / s_j (2D: h^2 / 4, 3D: h^2 / 8, powers of two, exact)
  for (int j = 1; j <= h->L; ++j) {
    Lev64& v = h->lv[j];
    const double sc = ND == 2 ? std::ldexp(1.0, -2 * j - 2) : std::ldexp(1.0, -2 * j - 3);
    hipLaunchKernelGGL(k64_scale<ND>, dim3(blocks_for(ND, v.n)), dim3(kF64Block), 0, s,
                       G64{v.n, v.pitch}, rhs[j - 1], v.b, sc);
  }
  // coarse levels: FMG 1..Lc in one launch
  hipLaunchKernelGGL(k64_coarse<ND>, dim3(1), dim3(kF64CoarseThreads), 0, s, h->lv_dev, 0, h->Lc,
                     h->c1, h->c2, h->c0, h->co, h->nu1, h->nu2, h->N, 0);
  for (int l = h->Lc + 1; l <= h->L; ++l) {
    Lev64& v = h->lv[l];
    Lev64& c = h->lv[l - 1];
    const G64 g{v.n, v.pitch};
    const unsigned nb = blocks_for(ND, v.n);
    hipLaunchKernelGGL(k64_prolong<ND>, dim3(nb), dim3(kF64Block), 0, s, G64{c.n, c.pitch}, g, c.x,
                       nullptr, v.x, 1.0, 0.0);
    for (int i = 0; i < h->N; ++i) {
      hipLaunchKernelGGL(k64_gemv<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.x, v.b, v.r, 1.0, -1.0,
                         h->c0, h->co);
      int rc = vcycle64<ND>(h, l, v.r, s);
      if (rc) return rc;
      hipLaunchKernelGGL(k64_sub<ND>, dim3(nb), dim3(kF64Block), 0, s, g, v.x, v.y, v.x);
    }
  }
  // x_out (dense (n+2)^ndim) = x_L
  Lev64& v = h->lv[h->L];
  const int64_t side = v.n + 2;
  const int64_t rows = ND == 3 ? side * side : side;
  return hip_check(hipMemcpy2DAsync(x_out, side * sizeof(double), v.x, v.pitch * sizeof(double),
                                    side * sizeof(double), rows, hipMemcpyDeviceToDevice, s),
                   "fp64 solution copy");
}

}  // namespace

extern "C" {

size_t fp64_mg_bytes(int ndim, int L) {
  if ((ndim != 2 && ndim != 3) || L < 1 || L > MG_MAX_LEVELS) return 0;
  fp64_mg tmp;
  return layout64(&tmp, ndim, L, nullptr);
}

int fp64_mg_create(int ndim, int L, int nu1, int nu2, int N, double c1, double c2, void* arena_dev,
                   size_t bytes, void* stream, fp64_mg** out) {
  if (!out || !arena_dev) return fail(BFP_EINVAL, "NULL argument");
  if ((ndim != 2 && ndim != 3) || L < 1 || L > MG_MAX_LEVELS)
    return fail(BFP_ESHAPE, "need ndim 2 or 3 and 1 <= L <= %d", MG_MAX_LEVELS);
  if (nu1 < 1 || nu2 < 0 || N < 1) return fail(BFP_EINVAL, "need nu1 >= 1, nu2 >= 0, N >= 1");
  if ((uintptr_t)arena_dev % 256) return fail(BFP_EINVAL, "arena must be 256-byte aligned");
  const size_t need = fp64_mg_bytes(ndim, L);
  if (bytes < need) return fail(BFP_ENOMEM, "arena holds %zu bytes, the FP64 solver needs %zu", bytes, need);
  fp64_mg* h = new (std::nothrow) fp64_mg();
  if (!h) return fail(BFP_ENOMEM, "host allocation failed");
  h->ndim = ndim;
  h->L = L;
  h->nu1 = nu1;
  h->nu2 = nu2;
  h->N = N;
  h->c1 = c1;
  h->c2 = c2;
  h->c0 = ndim == 2 ? 1.0 : 0.75;
  h->co = ndim == 2 ? -0.25 : -0.125;
  layout64(h, ndim, L, static_cast<char*>(arena_dev));
  h->Lc = 0;
  for (int j = 1; j <= L; ++j) {
    const int64_t n = h->lv[j].n;
    if ((ndim == 3 ? n * n * n : n * n) > kF64CoarsePts) break;
    h->Lc = j;
  }
  if (h->Lc == 0) h->Lc = 1;
  hipStream_t s = (hipStream_t)stream;
  int rc = hip_check(hipMemsetAsync(arena_dev, 0, need, s), "fp64 arena clear");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(h->lv_dev, h->lv, sizeof(Lev64) * (MG_MAX_LEVELS + 1),
                                  hipMemcpyHostToDevice, s), "fp64 level table");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "fp64 solver set-up");
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return BFP_OK;
}

int fp64_mg_fmg(fp64_mg* h, const double* const* rhs_dev, double* x_out_dev, void* stream) {
  if (!h || !rhs_dev || !x_out_dev) return fail(BFP_EINVAL, "NULL argument");
  for (int j = 0; j < h->L; ++j)
    if (!rhs_dev[j]) return fail(BFP_EINVAL, "right-hand side of level %d is NULL", j + 1);
  hipStream_t s = (hipStream_t)stream;
  return h->ndim == 2 ? fmg64<2>(h, rhs_dev, x_out_dev, s) : fmg64<3>(h, rhs_dev, x_out_dev, s);
}

int fp64_mg_destroy(fp64_mg* h) {
  delete h;
  return BFP_OK;
}

}  // extern "C"
