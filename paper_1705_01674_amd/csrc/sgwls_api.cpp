// C ABI of the SG-WLS library (declared in include/sgwls.h).
//
// Host-side validation, workspace layout and the order of passes of Sec. 2.3
// (T iterations of a column pass followed by a row pass).  All device memory
// is supplied by the caller; nothing here allocates.
#include "sgwls.h"
#include "sgwls_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

using namespace sgwls;

namespace {

constexpr int kVersion = 100;          // 0.1.0
constexpr int kMaxSide = 1 << 16;       // M, N limit (chunk grid dimension)
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

// Channel blocks: the kernels are compiled for 3 and 1 channels at a time.
int channel_block(int remaining) { return remaining >= 3 ? 3 : 1; }

// ---------------------------------------------------------------------------
// Tuning table: the kernel variant (rows per chunk, chunks per block) chosen
// for a pass, keyed by radius, channel block, precision, weight kind,
// direction and a size bucket (half-octaves of L*W).  Entries come from
// sgwls_autotune, sgwls_tune_pin or sgwls_tune_load; absent keys use
// variant 0.  Only stride-1 passes have variants.
using TuneKey = std::tuple<int, int, int, int, int, int>;
std::map<TuneKey, int>& tune_table() {
  static std::map<TuneKey, int> t;
  return t;
}
std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
int size_bucket(int L, int W) {
  return (int)std::lround(2.0 * std::log2((double)L * (double)W));
}
TuneKey tune_key(int r, int cb, int fp64, int kind, int dir, int L, int W) {
  return TuneKey(r, cb, fp64, kind, dir, size_bucket(L, W));
}
int tuned_variant(int r, int cb, int fp64, int kind, int dir, int L, int W) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  auto it = tune_table().find(tune_key(r, cb, fp64, kind, dir, L, W));
  return it == tune_table().end() ? 0 : it->second;
}

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
  wp.inv_sr2 = p.kind == SGWLS_W_EXP ? (float)(1.0 / ((double)p.sigma_r * p.sigma_r)) : 0.0f;
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

// Interface bytes needed by one pass direction over all channel blocks and
// all kernel variants (so a tuned variant never outgrows the workspace).
size_t pass_iface_bytes(int direction, int C, int M, int N, const sgwls_params& p) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  size_t need = 0;
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    need = std::max(need, interface_bytes_max(L, W, p.r, cb, p.stride, p.prec));
    c0 += cb;
  }
  return align_up(need);
}

size_t iface_bytes_all(int C, int M, int N, const sgwls_params& p) {
  return std::max(pass_iface_bytes(0, C, M, N, p), pass_iface_bytes(1, C, M, N, p));
}

size_t image_bytes(int C, int M, int N) { return align_up(sizeof(float) * (size_t)C * M * N); }

// variant < 0: the tuned variant of the case (variant 0 when none is tuned).
sgwls_status enqueue_pass(int direction, const float* x, const float* g, float* y, int C, int M,
                          int N, const sgwls_params& p, const float* lam_dev, void* iface,
                          hipStream_t stream, int stages = kStageAll, int variant = -1) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const WeightParams wp = weight_params(p);
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    const int v = variant >= 0 ? variant
                               : tuned_variant(p.r, cb, p.prec, (int)p.kind, direction, L, W);
    const PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec, v);
    const PassGeom geo = pass_geom(direction, M, N, pl, p.stride);
    hipError_t e = launch_pass(p.r, cb, p.prec, x, g, y, c0, geo, pl, wp, lam_dev, p.lambda,
                               iface, stream, stages);
    if (e != hipSuccess) return SGWLS_E_HIP;
    c0 += cb;
  }
  return SGWLS_OK;
}

// Backward workspace: the gradient ping-pong image, the interface buffers of
// the backward plans (two right-hand sides per channel), the side terms of
// chunk-boundary edges (P x W floats) and the per-block lambda partials.
struct BwdLayout {
  size_t img_off, iface_off, side_off, lpart_off, total;
};

BwdLayout bwd_layout(int C, int M, int N, const sgwls_params& p) {
  size_t iface = 0, side = 0, blocks = 0;
  for (int dir = 0; dir < 2; ++dir) {
    const int L = dir == 0 ? M : N, W = dir == 0 ? N : M;
    for (int c0 = 0; c0 < C;) {
      const int cb = channel_block(C - c0);
      iface = std::max(iface, interface_bytes_max(L, W, p.r, cb, p.stride, p.prec, kModeBackward));
      const VariantSet vs = variants_for(kModeBackward, p.r, cb, p.prec);
      for (int v = 0; v < (p.stride == 1 ? vs.n : 1); ++v) {
        const PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec, v, kModeBackward);
        const PassGeom geo = pass_geom(dir, M, N, pl, p.stride);
        side = std::max(side, (size_t)pl.P * W);
        blocks = std::max(blocks, (size_t)expand_blocks(geo, pl));
      }
      c0 += cb;
    }
  }
  BwdLayout l{};
  l.img_off = 0;
  l.iface_off = image_bytes(C, M, N);
  l.side_off = l.iface_off + align_up(iface);
  l.lpart_off = l.side_off + align_up(side * sizeof(float));
  l.total = l.lpart_off + align_up(blocks * sizeof(double));
  return l;
}

// One backward pass over all channel blocks.  `first` is true for the first
// launch of a backward call: it overwrites gbar and *grad_lambda, later
// launches add to them.
sgwls_status enqueue_pass_backward(int direction, const float* x, const float* g,
                                   const float* ybar, float* xbar, float* gbar,
                                   double* grad_lambda, int C, int M, int N,
                                   const sgwls_params& p, const float* lam_dev, void* ws,
                                   const BwdLayout& lay, hipStream_t stream, bool& first) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const WeightParams wp = weight_params(p);
  char* base = reinterpret_cast<char*>(ws);
  BwdArgs bw{};
  bw.ybar = ybar;
  bw.gbar = gbar;
  bw.side = reinterpret_cast<float*>(base + lay.side_off);
  bw.lpart = grad_lambda ? reinterpret_cast<double*>(base + lay.lpart_off) : nullptr;
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    const PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec, 0, kModeBackward);
    const PassGeom geo = pass_geom(direction, M, N, pl, p.stride);
    bw.gacc = first ? 0 : 1;
    hipError_t e = launch_pass(p.r, cb, p.prec, x, g, xbar, c0, geo, pl, wp, lam_dev, p.lambda,
                               base + lay.iface_off, stream, kStageAll, &bw);
    if (e != hipSuccess) return SGWLS_E_HIP;
    e = launch_bwd_fixup(bw.side, gbar, geo, bw.lpart, expand_blocks(geo, pl), grad_lambda,
                         first ? 0 : 1, stream);
    if (e != hipSuccess) return SGWLS_E_HIP;
    first = false;
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

int sgwls_variant_count(int r, int channel_block, int prec) {
  if (r < 1 || r > kMaxR || (channel_block != 1 && channel_block != 3) || (prec != 0 && prec != 1))
    return 0;
  return variants_of(r, channel_block, prec).n;
}

sgwls_status sgwls_tune_pin(int direction, int channel_block, int M, int N,
                            const sgwls_params* p, int variant) {
  sgwls_status st = sgwls_validate(channel_block, M, N, p);
  if (st != SGWLS_OK) return st;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if (channel_block != 1 && channel_block != 3) return SGWLS_E_ARG;
  if (variant < 0 || variant >= variants_of(p->r, channel_block, p->prec).n) return SGWLS_E_ARG;
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_table()[tune_key(p->r, channel_block, p->prec, (int)p->kind, direction, L, W)] = variant;
  return SGWLS_OK;
}

int sgwls_tune_query(int direction, int channel_block, int M, int N, const sgwls_params* p) {
  if (!p || (direction != 0 && direction != 1)) return -1;
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  return tuned_variant(p->r, channel_block, p->prec, (int)p->kind, direction, L, W);
}

void sgwls_tune_clear(void) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_table().clear();
}

int sgwls_tune_size(void) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  return (int)tune_table().size();
}

sgwls_status sgwls_autotune(const float* x, const float* g, float* y, int C, int M, int N,
                            const sgwls_params* p, void* ws, size_t ws_bytes, void* stream,
                            int reps, int* chosen) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (!x || !g || !y || y == x || (const float*)y == g || reps < 1) return SGWLS_E_ARG;
  const size_t need = std::max(pass_iface_bytes(0, C, M, N, *p), pass_iface_bytes(1, C, M, N, *p));
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  if (chosen)
    for (int i = 0; i < 4; ++i) chosen[i] = -1;
  if (p->stride != 1) return SGWLS_OK;   // strided passes have a single kernel
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SGWLS_E_HIP;
  }
  const WeightParams wp = weight_params(*p);
  sgwls_status result = SGWLS_OK;
  for (int dir = 0; dir < 2 && result == SGWLS_OK; ++dir) {
    const int L = dir == 0 ? M : N, W = dir == 0 ? N : M;
    for (int cbi = 0; cbi < 2 && result == SGWLS_OK; ++cbi) {
      const int cb = cbi == 0 ? 3 : 1;
      int c0 = -1;   // first channel block of this width
      for (int c = 0; c < C;) {
        const int b = channel_block(C - c);
        if (b == cb) { c0 = c; break; }
        c += b;
      }
      if (c0 < 0) continue;
      const int nv = variants_of(p->r, cb, p->prec).n;
      int best = 0;
      float best_ms = 0.0f;
      for (int v = 0; v < nv && result == SGWLS_OK; ++v) {
        const PassPlan pl = make_plan(L, W, p->r, cb, p->stride, p->prec, v);
        const PassGeom geo = pass_geom(dir, M, N, pl, p->stride);
        auto run = [&]() {
          return launch_pass(p->r, cb, p->prec, x, g, y, c0, geo, pl, wp, nullptr, p->lambda,
                             ws, s, kStageAll);
        };
        if (run() != hipSuccess || hipEventRecord(e0, s) != hipSuccess) { result = SGWLS_E_HIP; break; }
        for (int i = 0; i < reps; ++i)
          if (run() != hipSuccess) { result = SGWLS_E_HIP; break; }
        float ms = 0.0f;
        if (result != SGWLS_OK || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          result = SGWLS_E_HIP;
          break;
        }
        if (v == 0 || ms < best_ms) { best = v; best_ms = ms; }
      }
      if (result != SGWLS_OK) break;
      {
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_table()[tune_key(p->r, cb, p->prec, (int)p->kind, dir, L, W)] = best;
      }
      if (chosen) chosen[dir * 2 + cbi] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

sgwls_status sgwls_tune_save(const char* path, const char* arch) {
  if (!path || !arch || !arch[0] || std::strchr(arch, ' ') || std::strchr(arch, '\n'))
    return SGWLS_E_ARG;
  FILE* fp = std::fopen(path, "w");
  if (!fp) return SGWLS_E_ARG;
  std::lock_guard<std::mutex> lk(tune_mutex());
  std::fprintf(fp, "sgwls-tune %d %s\n", kVersion, arch);
  for (const auto& kv : tune_table()) {
    int r, cb, fp64, kind, dir, bucket;
    std::tie(r, cb, fp64, kind, dir, bucket) = kv.first;
    std::fprintf(fp, "%d %d %d %d %d %d %d\n", r, cb, fp64, kind, dir, bucket, kv.second);
  }
  const bool ok = std::fclose(fp) == 0;
  return ok ? SGWLS_OK : SGWLS_E_ARG;
}

sgwls_status sgwls_tune_load(const char* path, const char* arch) {
  if (!path || !arch) return SGWLS_E_ARG;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return SGWLS_E_ARG;
  char tag[32] = {0}, farch[128] = {0};
  int version = -1;
  std::map<TuneKey, int> entries;
  bool ok = std::fscanf(fp, "%31s %d %127s", tag, &version, farch) == 3 &&
            std::strcmp(tag, "sgwls-tune") == 0 && version == kVersion &&
            std::strcmp(farch, arch) == 0;
  while (ok) {
    int r, cb, fp64, kind, dir, bucket, v;
    const int got = std::fscanf(fp, "%d %d %d %d %d %d %d", &r, &cb, &fp64, &kind, &dir, &bucket, &v);
    if (got == EOF) break;
    if (got != 7 || r < 1 || r > kMaxR || (cb != 1 && cb != 3) || (fp64 != 0 && fp64 != 1) ||
        (kind != 0 && kind != 1) || (dir != 0 && dir != 1) || v < 0 ||
        v >= variants_of(r, cb, fp64).n) {
      ok = false;
      break;
    }
    entries[TuneKey(r, cb, fp64, kind, dir, bucket)] = v;
  }
  std::fclose(fp);
  if (!ok) return SGWLS_E_ARG;   // stale or corrupt: the table is left unchanged
  std::lock_guard<std::mutex> lk(tune_mutex());
  for (const auto& kv : entries) tune_table()[kv.first] = kv.second;
  return SGWLS_OK;
}

size_t sgwls_backward_workspace_bytes(int C, int M, int N, const sgwls_params* p) {
  if (sgwls_validate(C, M, N, p) != SGWLS_OK) return 0;
  return bwd_layout(C, M, N, *p).total;
}

sgwls_status sgwls_pass_backward(int direction, const float* x, const float* g,
                                 const float* ybar, float* xbar, float* gbar,
                                 double* grad_lambda, int C, int M, int N,
                                 const sgwls_params* p, const float* lambda_dev, void* ws,
                                 size_t ws_bytes, void* stream) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if (!x || !g || !ybar || !xbar || xbar == x || xbar == ybar || (const float*)xbar == g)
    return SGWLS_E_ARG;
  if (gbar && ((const float*)gbar == g || gbar == xbar || (const float*)gbar == x ||
               (const float*)gbar == ybar))
    return SGWLS_E_ARG;
  const BwdLayout lay = bwd_layout(C, M, N, *p);
  if (!ws || ws_bytes < lay.total) return SGWLS_E_WORKSPACE;
  bool first = true;
  return enqueue_pass_backward(direction, x, g, ybar, xbar, gbar, grad_lambda, C, M, N, *p,
                               lambda_dev, ws, lay, (hipStream_t)stream, first);
}

sgwls_status sgwls_backward(const float* g, const float* saved, const float* grad_u,
                            float* grad_f, float* grad_g, double* grad_lambda, int C, int M,
                            int N, const sgwls_params* p, const float* lambda_dev, void* ws,
                            size_t ws_bytes, void* stream) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (!g || !saved || !grad_u || !grad_f || (const float*)grad_f == g ||
      (const float*)grad_f == saved)
    return SGWLS_E_ARG;
  if (grad_g && ((const float*)grad_g == g || grad_g == grad_f || (const float*)grad_g == grad_u ||
                 (const float*)grad_g == saved))
    return SGWLS_E_ARG;
  const BwdLayout lay = bwd_layout(C, M, N, *p);
  if (!ws || ws_bytes < lay.total) return SGWLS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  float* tmp = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + lay.img_off);
  const size_t plane = (size_t)C * M * N;
  const int passes = 2 * p->iters;
  // Passes in reverse order.  Pass q reads the gradient of its output (grad_u
  // for the last pass) and writes that of its input: into grad_f for even q,
  // tmp for odd q, so pass 0 ends in grad_f and grad_u may alias grad_f.
  const float* ybar = grad_u;
  bool first = true;
  for (int q = passes - 1; q >= 0; --q) {
    float* xbar = (q % 2 == 0) ? grad_f : tmp;
    st = enqueue_pass_backward(q % 2, saved + (size_t)q * plane, g, ybar, xbar, grad_g,
                               grad_lambda, C, M, N, *p, lambda_dev, ws, lay, s, first);
    if (st != SGWLS_OK) return st;
    ybar = xbar;
  }
  return SGWLS_OK;
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
