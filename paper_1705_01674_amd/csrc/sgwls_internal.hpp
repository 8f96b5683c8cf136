// Internal declarations shared by the kernels (sgwls_kernels.hip) and the
// C ABI (sgwls_api.cpp).  Nothing here is part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sgwls {

constexpr int kMaxR = 4;     // largest neighbourhood radius compiled in
constexpr int kWave = 64;    // CDNA wavefront width

// Guidance-weight constants of Eq. (2), prepared on the host.
struct WeightParams {
  int kind;                    // 0: omega^exp, 1: omega^frac
  float spatial[kMaxR + 1];    // spatial factor S(d) for d = 1..r (index d)
  float range_c2;              // exp: log2(e) / (2 sigma_r^2), so R = 2^(-dG^2 * range_c2)
  float alpha_r;               // frac: exponent of |G_i - G_j|
  float eps;                   // frac: epsilon
};

// Geometry of one pass.  A pass solves one subsystem per strip centre k; the
// strip's rows (a = 0..L-1 along the pass) each contribute 2r+1 pixels
// (b = k-r..k+r across the pass).  Pixel (a, b) lives at a*sa + b*sb inside a
// channel plane, so the column pass has (L, W, sa, sb) = (M, N, N, 1) and the
// row pass (N, M, 1, N).
struct PassGeom {
  int L;            // rows along the pass (subsystem length / (2r+1))
  int W;            // extent across the pass (strip centres lie in [r, W-1-r])
  long long sa, sb; // strides of the along / across coordinates
  long long plane;  // M*N, the stride between channel planes
  int nK;           // number of strip centres
  int stride;       // sliding step tau between centres
  int R;            // rows per chunk (the partition of every subsystem)
  int P;            // chunks per subsystem = ceil(L / R)
};

// Launch configuration of one (r, channel block, precision, stride) case.
struct PassPlan {
  int R;            // rows per chunk
  int Q;            // chunks per reduce / expand block (one wave each)
  int P;            // chunks per subsystem
  int nK;           // strip centres
  int OW;           // output columns owned by one expand block
  int TB;           // LDS tile width (columns across the pass)
  int pitch;        // LDS row pitch (odd)
  int iface_m;      // separators per lane of the wave interface solver (0: serial solver)
  size_t sum_elems, u_elems;   // interface buffer sizes (elements)
  int acc_bytes;    // 4 (float) or 8 (double) interface element size
};

// Host-side helpers (sgwls_kernels.hip).
int strip_count(int W, int r, int stride);
PassPlan make_plan(int L, int W, int r, int cb, int stride, int fp64);
size_t interface_bytes(const PassPlan& pl);

// Stages of one pass (bit mask): reduce, interface solve, expand.
constexpr int kStageReduce = 1, kStageInterface = 2, kStageExpand = 4, kStageAll = 7;

// Enqueue the stages in `stages` of one pass for channels [c0, c0+cb) of x
// into y.  `iface` must hold interface_bytes(plan).  Returns a hipError_t.
hipError_t launch_pass(int r, int cb, int fp64, const float* x, const float* g, float* y,
                       int c0, const PassGeom& geo, const PassPlan& plan,
                       const WeightParams& wp, const float* lam_dev, float lam_host,
                       void* iface, hipStream_t stream, int stages);

}  // namespace sgwls
