// C ABI of the SG-WLS library (declared in include/sgwls.h).
//
// Host-side validation, workspace layout and the order of passes of Sec. 2.3
// (T iterations of a column pass followed by a row pass).  All device memory
// is supplied by the caller; nothing here allocates.
#include "sgwls.h"
#include "sgwls_internal.hpp"

#include <algorithm>
#include <cmath>

using namespace sgwls;

namespace {

constexpr int kVersion = 100;          // 0.1.0
constexpr int kMaxSide = 1 << 16;       // M, N limit (chunk grid dimension)
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

// Channel blocks: the kernels are compiled for 3 and 1 channels at a time.
int channel_block(int remaining) { return remaining >= 3 ? 3 : 1; }

WeightParams weight_params(const sgwls_params& p) {
  WeightParams wp{};
  wp.kind = (int)p.kind;
  for (int d = 0; d <= kMaxR; ++d) {
    double s = 0.0;
    if (d >= 1) {
      if (p.kind == SGWLS_W_EXP)
        s = std::exp(-(double)d * d / (2.0 * (double)p.sigma_s * p.sigma_s));
      else
        s = 1.0 / (std::pow((double)d, (double)p.alpha_s) + (double)p.eps);
    }
    wp.spatial[d] = (float)s;
  }
  // exp range factor as a power of two: exp(-x) = 2^(-x log2(e))
  wp.range_c2 = p.kind == SGWLS_W_EXP
                    ? (float)(1.4426950408889634 / (2.0 * (double)p.sigma_r * p.sigma_r))
                    : 0.0f;
  wp.alpha_r = p.alpha_r;
  wp.eps = p.eps;
  return wp;
}

PassGeom pass_geom(int direction, int M, int N, const PassPlan& pl, int stride) {
  PassGeom g{};
  if (direction == 0) {
    g.L = M; g.W = N; g.sa = N; g.sb = 1;
  } else {
    g.L = N; g.W = M; g.sa = 1; g.sb = N;
  }
  g.plane = (long long)M * N;
  g.nK = pl.nK;
  g.stride = stride;
  g.R = pl.R;
  g.P = pl.P;
  return g;
}

// Interface bytes needed by one pass direction over all channel blocks.
size_t pass_iface_bytes(int direction, int C, int M, int N, const sgwls_params& p) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  size_t need = 0;
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    need = std::max(need, interface_bytes(make_plan(L, W, p.r, cb, p.stride, p.prec)));
    c0 += cb;
  }
  return align_up(need);
}

size_t iface_bytes_all(int C, int M, int N, const sgwls_params& p) {
  return std::max(pass_iface_bytes(0, C, M, N, p), pass_iface_bytes(1, C, M, N, p));
}

size_t image_bytes(int C, int M, int N) { return align_up(sizeof(float) * (size_t)C * M * N); }

sgwls_status enqueue_pass(int direction, const float* x, const float* g, float* y, int C, int M,
                          int N, const sgwls_params& p, const float* lam_dev, void* iface,
                          hipStream_t stream, int stages = kStageAll) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const WeightParams wp = weight_params(p);
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    const PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec);
    const PassGeom geo = pass_geom(direction, M, N, pl, p.stride);
    hipError_t e = launch_pass(p.r, cb, p.prec, x, g, y, c0, geo, pl, wp, lam_dev, p.lambda,
                               iface, stream, stages);
    if (e != hipSuccess) return SGWLS_E_HIP;
    c0 += cb;
  }
  return SGWLS_OK;
}

}  // namespace

extern "C" {

const char* sgwls_status_str(sgwls_status s) {
  switch (s) {
    case SGWLS_OK: return "ok";
    case SGWLS_E_ARG: return "invalid argument";
    case SGWLS_E_SHAPE: return "invalid shape";
    case SGWLS_E_WORKSPACE: return "workspace missing or too small";
    case SGWLS_E_UNSUPPORTED: return "unsupported by this build";
    case SGWLS_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

int sgwls_version(void) { return kVersion; }

sgwls_status sgwls_validate(int C, int M, int N, const sgwls_params* p) {
  if (!p) return SGWLS_E_ARG;
  if (p->r < 1 || p->iters < 1) return SGWLS_E_ARG;
  if (p->stride < 1 || p->stride > 2 * p->r + 1) return SGWLS_E_ARG;
  if (!std::isfinite(p->lambda) || p->lambda < 0.0f) return SGWLS_E_ARG;
  if (p->kind == SGWLS_W_EXP) {
    if (!finite_pos(p->sigma_s) || !finite_pos(p->sigma_r)) return SGWLS_E_ARG;
  } else if (p->kind == SGWLS_W_FRAC) {
    if (!std::isfinite(p->alpha_s) || p->alpha_s < 0.0f) return SGWLS_E_ARG;
    if (!std::isfinite(p->alpha_r) || p->alpha_r < 0.0f) return SGWLS_E_ARG;
    if (!finite_pos(p->eps)) return SGWLS_E_ARG;
  } else {
    return SGWLS_E_ARG;
  }
  if (p->prec != SGWLS_P_FP32 && p->prec != SGWLS_P_FP64_PIVOT) return SGWLS_E_ARG;
  if (C < 1 || M < 2 * p->r + 1 || N < 2 * p->r + 1) return SGWLS_E_SHAPE;
  // kernels address pixels with 32-bit element offsets
  if (M > kMaxSide || N > kMaxSide || (long long)C * M * N > 0x7fffffffLL) return SGWLS_E_SHAPE;
  if (p->r > kMaxR) return SGWLS_E_UNSUPPORTED;
  return SGWLS_OK;
}

size_t sgwls_workspace_bytes(int C, int M, int N, const sgwls_params* p) {
  if (sgwls_validate(C, M, N, p) != SGWLS_OK) return 0;
  return image_bytes(C, M, N) + iface_bytes_all(C, M, N, *p);
}

sgwls_status sgwls_pass_stages(int stages, int direction, const float* x, const float* g,
                               float* y, int C, int M, int N, const sgwls_params* p,
                               const float* lambda_dev, void* ws, size_t ws_bytes,
                               void* stream) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if (stages < 1 || stages > kStageAll) return SGWLS_E_ARG;
  if (!x || !g || !y || y == x || (const float*)y == g) return SGWLS_E_ARG;
  const size_t need = pass_iface_bytes(direction, C, M, N, *p);
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  return enqueue_pass(direction, x, g, y, C, M, N, *p, lambda_dev, ws, (hipStream_t)stream,
                      stages);
}

sgwls_status sgwls_pass(int direction, const float* x, const float* g, float* y, int C, int M,
                        int N, const sgwls_params* p, const float* lambda_dev, void* ws,
                        size_t ws_bytes, void* stream) {
  return sgwls_pass_stages(kStageAll, direction, x, g, y, C, M, N, p, lambda_dev, ws, ws_bytes,
                           stream);
}

sgwls_status sgwls_filter(const float* f, const float* g, float* u, int C, int M, int N,
                          const sgwls_params* p, const float* lambda_dev, float* saved,
                          void* ws, size_t ws_bytes, void* stream) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (!f || !g || !u || (const float*)u == g) return SGWLS_E_ARG;
  const size_t img = image_bytes(C, M, N);
  const size_t need = img + iface_bytes_all(C, M, N, *p);
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  float* tmp = reinterpret_cast<float*>(ws);
  void* iface = reinterpret_cast<char*>(ws) + img;
  const size_t plane = (size_t)C * M * N;
  const int passes = 2 * p->iters;
  // Pass q reads x_q and writes x_{q+1}; x_0 = f and x_{2T} = u.  With saved,
  // x_q lives in saved[q] (q < 2T); otherwise passes ping-pong between tmp
  // and u so that the last one lands in u.
  if (saved) {
    if (hipMemcpyAsync(saved, f, sizeof(float) * plane, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return SGWLS_E_HIP;
  }
  const float* x = saved ? saved : f;
  for (int q = 0; q < passes; ++q) {
    float* y;
    if (q == passes - 1) y = u;
    else if (saved) y = saved + (size_t)(q + 1) * plane;
    else y = ((passes - q) % 2 == 0) ? tmp : u;
    st = enqueue_pass(q % 2, x, g, y, C, M, N, *p, lambda_dev, iface, s);
    if (st != SGWLS_OK) return st;
    x = y;
  }
  return SGWLS_OK;
}

size_t sgwls_backward_workspace_bytes(int C, int M, int N, const sgwls_params* p) {
  (void)C; (void)M; (void)N; (void)p;
  return 0;
}

sgwls_status sgwls_backward(const float* g, const float* saved, const float* grad_u,
                            float* grad_f, float* grad_g, double* grad_lambda, int C, int M,
                            int N, const sgwls_params* p, const float* lambda_dev, void* ws,
                            size_t ws_bytes, void* stream) {
  (void)g; (void)saved; (void)grad_u; (void)grad_f; (void)grad_g; (void)grad_lambda;
  (void)C; (void)M; (void)N; (void)p; (void)lambda_dev; (void)ws; (void)ws_bytes; (void)stream;
  return SGWLS_E_UNSUPPORTED;
}

size_t sgwls_batched_workspace_bytes(const sgwls_image* imgs, const sgwls_params* p, int B) {
  (void)imgs; (void)p; (void)B;
  return 0;
}

sgwls_status sgwls_filter_batched(const sgwls_image* imgs, const sgwls_params* p, int B,
                                  void* ws, size_t ws_bytes, void* stream) {
  (void)imgs; (void)p; (void)B; (void)ws; (void)ws_bytes; (void)stream;
  return SGWLS_E_UNSUPPORTED;
}

}  // extern "C"
