// Host-side planning of a pass: chunking, block geometry, interface buffers,
// and dispatch to the per-radius kernel translation units.
#include "sgwls_internal.hpp"

#include <algorithm>

namespace sgwls {

int strip_count(int W, int r, int stride) {
  if (r < 1 || stride < 1 || W < 2 * r + 1) return 0;
  const int span = W - 1 - 2 * r;          // offset of the last regular centre
  const int regular = span / stride + 1;
  return regular + ((span % stride) != 0 ? 1 : 0);
}

PassPlan make_plan(int L, int W, int r, int cb, int stride, int fp64, int variant, int mode) {
  PassPlan pl{};
  const VariantSet vs = variants_for(mode, r, cb, fp64);
  if (variant < 0 || variant >= (stride == 1 ? vs.n : strided_variant_count(r, cb, fp64, mode)))
    variant = 0;
  if (stride != 1 && variant > 0) {
    // LDS accumulators of the strided expand: cb planes of Q R + 2 rows
    const StridedVariant sv = strided_variant(r, cb, fp64, variant);
    const int pitch = ((kWave - 1) * stride + 2 * r + 1) | 1;
    if (sizeof(float) * (size_t)cb * (sv.Q * sv.R + 2) * pitch > kStridedLdsMax) variant = 0;
  }
  pl.mode = mode;
  pl.nr = mode == kModeBackward ? 2 * cb : cb;
  pl.variant = variant;
  if (stride == 1) {
    pl.R = vs.v[variant].R;
    pl.Q = vs.v[variant].Q;
  } else if (variant == 0) {   // the mode's own variant 0 (backward chunks differ)
    pl.R = vs.v[0].R;
    pl.Q = 1;
  } else {
    const StridedVariant sv = strided_variant(r, cb, fp64, variant);
    pl.R = sv.R;
    pl.Q = sv.Q;
  }
  pl.P = (L + pl.R - 1) / pl.R;
  pl.nK = strip_count(W, r, stride);
  pl.OW = stride == 1 ? kWave - 2 * r : (kWave - 2) * stride - 2 * r;
  pl.TB = stride == 1 ? kWave + 2 * r : (kWave - 1) * stride + 2 * r + 1;
  pl.pitch = pl.TB | 1;
  const int n = pl.P - 1;
  const int m = (n + kWave - 1) / kWave;
  pl.iface_m = (vs.MM > 0 && m <= vs.MM) ? std::max(m, 1) : 0;
  const int T2 = r * (r + 1) / 2;
  const int F = 2 * T2 + 2 * r * pl.nr + r * r;
  pl.acc_bytes = fp64 ? 8 : 4;
  pl.one = nullptr;
  pl.us_out = nullptr;
  pl.sum_elems = (size_t)pl.P * F * pl.nK;
  pl.u_elems = (size_t)std::max(n, 1) * r * pl.nr * pl.nK;
  // Runs longer than the register solver holds go to the long-run solver,
  // whose per-block values (3r^2 + r*nr each, m blocks per lane, NL lanes
  // per strip) live in scratch after the separator solutions.  NL: one wave
  // per strip, or four or two where that still gives at most 2048 waves (the
  // strips alone leave the GPU underfilled; their runs shorten by as much)
  // and the exchange fits 64 KiB of LDS.  Measured at 1024x1024 RGB, r = 4:
  // stride 4 0.97 -> 0.80 ms, stride 9 0.85 -> 0.66 ms; at stride 1 with more
  // strips than that a single wave per strip is as fast or faster.
  // Float32 forward passes at r = 3: the register solver on 128 or 256 lanes
  // per strip (at most 4 blocks per lane, no scratch) where that holds the
  // runs (lines up to 1025 chunks).
  pl.mw_nl = 0;
  if (n > 0 && pl.iface_m == 0 && r == 3 && !fp64 && mode == kModeForward) {
    for (int nl : {2 * kWave, 4 * kWave})
      if (n <= 4 * nl) {
        pl.mw_nl = nl;
        break;
      }
  }
  pl.long_nl = kWave;
  if (n > 0 && pl.iface_m == 0) {
    const size_t slot = (size_t)(3 * r * r + r * pl.nr) * pl.acc_bytes;
    for (int nw : {4, 2}) {
      if ((long long)pl.nK * nw <= 2048 && (size_t)nw * kWave * slot <= 65536 && n > nw * kWave) {
        pl.long_nl = nw * kWave;
        break;
      }
    }
  }
  const int ml = (n + pl.long_nl - 1) / pl.long_nl;
  pl.g_elems = (n > 0 && pl.iface_m == 0)
                   ? (size_t)std::max(ml, 1) * pl.long_nl * (3 * r * r + r * pl.nr) * pl.nK
                   : 0;
  return pl;
}

size_t interface_bytes(const PassPlan& pl) {
  // chunk summaries, separator solutions, long-run solver scratch
  return (pl.sum_elems + pl.u_elems + pl.g_elems) * (size_t)pl.acc_bytes + 256;
}

size_t interface_bytes_max(int L, int W, int r, int cb, int stride, int fp64, int mode) {
  const VariantSet vs = variants_for(mode, r, cb, fp64);
  size_t need = 0;
  const int nv = stride == 1 ? vs.n : strided_variant_count(r, cb, fp64, mode);
  for (int v = 0; v < nv; ++v)
    need = std::max(need, interface_bytes(make_plan(L, W, r, cb, stride, fp64, v, mode)));
  return need;
}

bool frames_supported(int C, int r, int stride, int fp64) {
  if (stride != 1 || r < 1 || r > kMaxR) return false;
  const int cbs[2] = {3, 1};
  for (int cb : cbs) {
    if (cb == 3 && C < 3) continue;
    if (cb == 1 && C % 3 == 0) continue;
    if (!variants_of(r, cb, fp64).v[0].D || !bwd_variants_of(r, cb, fp64).v[0].D) return false;
  }
  return true;
}

int expand_blocks(const PassGeom& geo, const PassPlan& pl) {
  return ((geo.W + pl.OW - 1) / pl.OW) * ((geo.P + pl.Q - 1) / pl.Q);
}

hipError_t launch_pass(int r, int cb, int fp64, const float* x, const float* g, float* y,
                       int c0, const PassGeom& geo, const PassPlan& plan,
                       const WeightParams& wp, const float* lam_dev, float lam_host,
                       void* iface, hipStream_t stream, int st, const BwdArgs* bw) {
  if (plan.mode == kModeBackward && !bw) return hipErrorInvalidValue;
  if (plan.mode == kModeAdjoint && (st & kStageExpand)) return hipErrorInvalidValue;
  switch (r) {
    case 1: return launch_pass_r1(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st, bw);
    case 2: return launch_pass_r2(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st, bw);
    case 3: return launch_pass_r3(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st, bw);
    case 4: return launch_pass_r4(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st, bw);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sgwls
