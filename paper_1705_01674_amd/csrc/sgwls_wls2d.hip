// Reference solver of the 2D WLS model that SG-WLS approximates (Eqs. 1-4):
// (I + lambda L) u = f, where L couples every pixel with the (2r+1) x (2r+1)
// patch around it with the weights of Eq. 2 (|i - j| the Euclidean distance
// of the two pixels).  Jacobi-preconditioned conjugate gradients, one CG per
// channel, all channels in every launch; the matrix is never stored (the
// weights are recomputed from g in every product).  Dot products are float64
// and reduced in a fixed order, so a run is reproducible.
#include <cmath>
#include <vector>

#include "sgwls.h"
#include "sgwls_device.hpp"

namespace sgwls {
namespace {

constexpr int kCgTile = 16;                          // 16 x 16 pixels per workgroup
constexpr int kCgThreads = kCgTile * kCgTile;
constexpr int kCgMaxC = 4;
constexpr int kPatchMax = (2 * kMaxR + 1) * (2 * kMaxR + 1);

// lambda * spatial factor of every patch offset (dy, dx), index
// (dy + r) * (2r + 1) + (dx + r); the centre entry is unused.
struct Patch {
  int r;
  float ls[kPatchMax];
};

struct CgScalars {   // per channel
  double rz[kCgMaxC], alpha[kCgMaxC], beta[kCgMaxC], rr[kCgMaxC], ff[kCgMaxC];
};

// Fixed-order block sum of v over kCgThreads threads (result on thread 0).
DEV double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kCgThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

DEV int block_linear() { return blockIdx.y * gridDim.x + blockIdx.x; }

// d = diag(A) = 1 + lambda * sum_j omega_ij.
template <int KIND>
__global__ __launch_bounds__(kCgThreads) void k_cg_diag(const float* __restrict__ g,
                                                        float* __restrict__ d, int M, int N,
                                                        Patch pt, WeightParams wp) {
  const int x = blockIdx.x * kCgTile + threadIdx.x % kCgTile;
  const int y = blockIdx.y * kCgTile + threadIdx.x / kCgTile;
  if (x >= N || y >= M) return;
  const int r = pt.r, w = 2 * r + 1;
  const float gi = g[(size_t)y * N + x];
  float s = 1.0f;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      const int yy = y + dy, xx = x + dx;
      if ((dy | dx) == 0 || yy < 0 || yy >= M || xx < 0 || xx >= N) continue;
      s += pt.ls[(dy + r) * w + dx + r] * range_weight<KIND>(gi - g[(size_t)yy * N + xx], wp);
    }
  d[(size_t)y * N + x] = s;
}

// u = 0, r = f, z = f / d, p_old = 0; partials of (f.z, f.f) per channel.
__global__ __launch_bounds__(kCgThreads) void k_cg_init(const float* __restrict__ f,
                                                        const float* __restrict__ d,
                                                        float* __restrict__ u,
                                                        float* __restrict__ res,
                                                        float* __restrict__ z,
                                                        float* __restrict__ pold, int C, int M,
                                                        int N, double* __restrict__ part) {
  __shared__ double red[kCgThreads];
  const int x = blockIdx.x * kCgTile + threadIdx.x % kCgTile;
  const int y = blockIdx.y * kCgTile + threadIdx.x / kCgTile;
  const bool in = x < N && y < M;
  const size_t plane = (size_t)M * N, i = (size_t)y * N + x;
  for (int c = 0; c < C; ++c) {
    double fz = 0.0, ff = 0.0;
    if (in) {
      const float fv = f[c * plane + i];
      const float zv = fv / d[i];
      u[c * plane + i] = 0.0f;
      res[c * plane + i] = fv;
      z[c * plane + i] = zv;
      pold[c * plane + i] = 0.0f;
      fz = double(fv) * zv;
      ff = double(fv) * fv;
    }
    fz = block_sum(fz, red);
    ff = block_sum(ff, red);
    if (threadIdx.x == 0) {
      part[((size_t)block_linear() * C + c) * 2 + 0] = fz;
      part[((size_t)block_linear() * C + c) * 2 + 1] = ff;
    }
  }
}

// p = z + beta p_old (written to pnew) and q = A p; partials of p.q.
template <int KIND>
__global__ __launch_bounds__(kCgThreads) void k_cg_apply(
    const float* __restrict__ g, const float* __restrict__ z, const float* __restrict__ pold,
    float* __restrict__ pnew, float* __restrict__ q, const CgScalars* __restrict__ sc, int C,
    int M, int N, Patch pt, WeightParams wp, double* __restrict__ part) {
  __shared__ double red[kCgThreads];
  const int x = blockIdx.x * kCgTile + threadIdx.x % kCgTile;
  const int y = blockIdx.y * kCgTile + threadIdx.x / kCgTile;
  const bool in = x < N && y < M;
  const size_t plane = (size_t)M * N, i = (size_t)y * N + x;
  const int r = pt.r, w = 2 * r + 1;
  float beta[kCgMaxC], pi[kCgMaxC], acc[kCgMaxC];
  for (int c = 0; c < C; ++c) {
    beta[c] = float(sc->beta[c]);
    pi[c] = in ? z[c * plane + i] + beta[c] * pold[c * plane + i] : 0.0f;
    acc[c] = pi[c];
  }
  if (in) {
    const float gi = g[i];
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const int yy = y + dy, xx = x + dx;
        if ((dy | dx) == 0 || yy < 0 || yy >= M || xx < 0 || xx >= N) continue;
        const size_t j = (size_t)yy * N + xx;
        const float lw = pt.ls[(dy + r) * w + dx + r] * range_weight<KIND>(gi - g[j], wp);
        for (int c = 0; c < C; ++c) {
          const float pj = z[c * plane + j] + beta[c] * pold[c * plane + j];
          acc[c] += lw * (pi[c] - pj);
        }
      }
    for (int c = 0; c < C; ++c) {
      pnew[c * plane + i] = pi[c];
      q[c * plane + i] = acc[c];
    }
  }
  for (int c = 0; c < C; ++c) {
    const double pq = block_sum(in ? double(pi[c]) * acc[c] : 0.0, red);
    if (threadIdx.x == 0) part[(size_t)block_linear() * C + c] = pq;
  }
}

// u += alpha p, r -= alpha q, z = r / d; partials of (r.z, r.r).
__global__ __launch_bounds__(kCgThreads) void k_cg_update(
    float* __restrict__ u, float* __restrict__ res, float* __restrict__ z,
    const float* __restrict__ p, const float* __restrict__ q, const float* __restrict__ d,
    const CgScalars* __restrict__ sc, int C, int M, int N, double* __restrict__ part) {
  __shared__ double red[kCgThreads];
  const int x = blockIdx.x * kCgTile + threadIdx.x % kCgTile;
  const int y = blockIdx.y * kCgTile + threadIdx.x / kCgTile;
  const bool in = x < N && y < M;
  const size_t plane = (size_t)M * N, i = (size_t)y * N + x;
  for (int c = 0; c < C; ++c) {
    double rz = 0.0, rr = 0.0;
    if (in) {
      const float a = float(sc->alpha[c]);
      u[c * plane + i] += a * p[c * plane + i];
      const float rv = res[c * plane + i] - a * q[c * plane + i];
      const float zv = rv / d[i];
      res[c * plane + i] = rv;
      z[c * plane + i] = zv;
      rz = double(rv) * zv;
      rr = double(rv) * rv;
    }
    rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
      part[((size_t)block_linear() * C + c) * 2 + 0] = rz;
      part[((size_t)block_linear() * C + c) * 2 + 1] = rr;
    }
  }
}

// One workgroup: fixed-order sums of the block partials, then the scalars.
// mode 0 (after k_cg_init): rz = sum f.z, ff = sum f.f, beta = 0.
// mode 1 (after k_cg_apply): alpha = rz / sum p.q (0 when p.q is 0).
// mode 2 (after k_cg_update): beta = sum r.z / rz, rz = sum r.z, rr = sum r.r.
__global__ __launch_bounds__(kCgThreads) void k_cg_scalars(const double* __restrict__ part,
                                                           int nblocks, int C, int mode,
                                                           CgScalars* __restrict__ sc) {
  __shared__ double red[kCgThreads];
  const int stride = mode == 1 ? 1 : 2;
  for (int c = 0; c < C; ++c) {
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += kCgThreads) {
      a += part[((size_t)k * C + c) * stride];
      if (stride == 2) b += part[((size_t)k * C + c) * 2 + 1];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
      if (mode == 0) {
        sc->rz[c] = a;
        sc->ff[c] = b;
        sc->rr[c] = b;
        sc->beta[c] = 0.0;
      } else if (mode == 1) {
        sc->alpha[c] = a != 0.0 ? sc->rz[c] / a : 0.0;
      } else {
        sc->beta[c] = sc->rz[c] != 0.0 ? a / sc->rz[c] : 0.0;
        sc->rz[c] = a;
        sc->rr[c] = b;
      }
    }
  }
}

struct CgLayout {
  size_t res, z, pa, pb, q, d, part, sc, total;
};

// The range factor's parameters (Eq. 2) in the form range_weight reads.
WeightParams range_params(const sgwls_params& p) {
  WeightParams wp{};
  wp.kind = (int)p.kind;
  wp.range_c2 = p.kind == SGWLS_W_EXP
                    ? (float)(1.4426950408889634 / (2.0 * (double)p.sigma_r * p.sigma_r))
                    : 0.0f;
  wp.alpha_r = p.alpha_r;
  wp.eps = p.eps;
  return wp;
}

CgLayout cg_layout(int C, int M, int N) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t img = al(sizeof(float) * (size_t)C * M * N);
  const size_t nb = (size_t)((N + kCgTile - 1) / kCgTile) * ((M + kCgTile - 1) / kCgTile);
  CgLayout l{};
  l.res = 0;
  l.z = l.res + img;
  l.pa = l.z + img;
  l.pb = l.pa + img;
  l.q = l.pb + img;
  l.d = l.q + img;
  l.part = l.d + al(sizeof(float) * (size_t)M * N);
  l.sc = l.part + al(sizeof(double) * nb * C * 2);
  l.total = l.sc + al(sizeof(CgScalars));
  return l;
}

}  // namespace
}  // namespace sgwls

using namespace sgwls;

extern "C" {

namespace {
// The 2D model uses lambda, r and the weights only: the precision field is
// not validated against r.
sgwls_status validate_model(int C, int M, int N, const sgwls_params* p) {
  if (!p) return SGWLS_E_ARG;
  sgwls_params q = *p;
  q.prec = SGWLS_P_FP32;
  return sgwls_validate(C, M, N, &q);
}
}  // namespace

size_t sgwls_wls2d_workspace_bytes(int C, int M, int N, const sgwls_params* p) {
  if (C < 1 || C > kCgMaxC || validate_model(C, M, N, p) != SGWLS_OK) return 0;
  return cg_layout(C, M, N).total;
}

sgwls_status sgwls_wls2d(const float* f, const float* g, float* u, int C, int M, int N,
                         const sgwls_params* p, int max_iters, double tol, int* iters_done,
                         double* rel_residual, void* ws, size_t ws_bytes, void* stream) {
  if (C < 1 || C > kCgMaxC) return SGWLS_E_ARG;
  sgwls_status st = validate_model(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (!f || !g || !u || (const float*)u == g || max_iters < 1 || !(tol >= 0.0))
    return SGWLS_E_ARG;
  const CgLayout l = cg_layout(C, M, N);
  if (!ws || ws_bytes < l.total) return SGWLS_E_WORKSPACE;
  (void)hipGetLastError();   // report only this call's launch errors
  hipStream_t s = (hipStream_t)stream;
  char* base = reinterpret_cast<char*>(ws);
  float* res = reinterpret_cast<float*>(base + l.res);
  float* z = reinterpret_cast<float*>(base + l.z);
  float* pa = reinterpret_cast<float*>(base + l.pa);
  float* pb = reinterpret_cast<float*>(base + l.pb);
  float* q = reinterpret_cast<float*>(base + l.q);
  float* d = reinterpret_cast<float*>(base + l.d);
  double* part = reinterpret_cast<double*>(base + l.part);
  CgScalars* sc = reinterpret_cast<CgScalars*>(base + l.sc);

  // lambda * spatial factor per patch offset, from Eq. 2 at the Euclidean
  // distance of the offset.
  const int r = p->r, w = 2 * r + 1;
  Patch pt{};
  pt.r = r;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      const double dist = std::sqrt(double(dy * dy + dx * dx));
      double sp = 0.0;
      if (dy != 0 || dx != 0)
        sp = p->kind == SGWLS_W_EXP
                 ? std::exp(-dist * dist / (2.0 * double(p->sigma_s) * p->sigma_s))
                 : 1.0 / (std::pow(dist, double(p->alpha_s)) + double(p->eps));
      pt.ls[(dy + r) * w + dx + r] = float(double(p->lambda) * sp);
    }
  const WeightParams wp = range_params(*p);
  const dim3 grid((N + kCgTile - 1) / kCgTile, (M + kCgTile - 1) / kCgTile);
  const int nb = (int)(grid.x * grid.y);
  const bool frac = p->kind == SGWLS_W_FRAC;
  if (frac)
    hipLaunchKernelGGL(k_cg_diag<1>, grid, dim3(kCgThreads), 0, s, g, d, M, N, pt, wp);
  else
    hipLaunchKernelGGL(k_cg_diag<0>, grid, dim3(kCgThreads), 0, s, g, d, M, N, pt, wp);
  hipLaunchKernelGGL(k_cg_init, grid, dim3(kCgThreads), 0, s, f, d, u, res, z, pa, C, M, N, part);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kCgThreads), 0, s, part, nb, C, 0, sc);
  if (hipGetLastError() != hipSuccess) return SGWLS_E_HIP;
  // Convergence: max over channels of ||r|| / ||f|| <= tol, checked every
  // kCheck iterations (one stream synchronisation each).
  constexpr int kCheck = 8;
  CgScalars host{};
  int it = 0;
  double rel = 1.0;
  float* pold = pa;
  float* pnew = pb;
  while (it < max_iters) {
    if (frac)
      hipLaunchKernelGGL(k_cg_apply<1>, grid, dim3(kCgThreads), 0, s, g, z, pold, pnew, q, sc, C,
                         M, N, pt, wp, part);
    else
      hipLaunchKernelGGL(k_cg_apply<0>, grid, dim3(kCgThreads), 0, s, g, z, pold, pnew, q, sc, C,
                         M, N, pt, wp, part);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kCgThreads), 0, s, part, nb, C, 1, sc);
    hipLaunchKernelGGL(k_cg_update, grid, dim3(kCgThreads), 0, s, u, res, z, pnew, q, d, sc, C,
                       M, N, part);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kCgThreads), 0, s, part, nb, C, 2, sc);
    if (hipGetLastError() != hipSuccess) return SGWLS_E_HIP;
    std::swap(pold, pnew);
    ++it;
    if (it % kCheck == 0 || it == max_iters) {
      if (hipMemcpyAsync(&host, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return SGWLS_E_HIP;
      rel = 0.0;
      for (int c = 0; c < C; ++c)
        rel = std::max(rel, host.ff[c] > 0.0 ? std::sqrt(host.rr[c] / host.ff[c]) : 0.0);
      if (rel <= tol) break;
    }
  }
  if (iters_done) *iters_done = it;
  if (rel_residual) *rel_residual = rel;
  return SGWLS_OK;
}

}  // extern "C"
