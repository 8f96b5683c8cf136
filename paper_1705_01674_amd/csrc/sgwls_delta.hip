// Cancellation-free float32 precision mode for r = 1 (SGWLS_P_FP32_DELTA).
//
// At r = 1 every subsystem A = I + lambda L of a strip (Eq. 4) is
// tridiagonal: element p of the snake (Sec. 2.1) couples to p + 1 with
// c_p = lambda w_p.  The banded LDL^T of Sec. 2.2 takes the pivots
// alpha_p = (1 + c_{p-1} + c_p) - c_{p-1}^2 / alpha_{p-1}; when lambda w is
// large the 1 that keeps A well conditioned is below float32 resolution of
// that difference and is lost.  Here each pivot is carried as its excess
// over the coupling still to be eliminated, delta_p = alpha_p - c_p:
//   delta_0 = 1,  delta_{p+1} = 1 + c_p delta_p / alpha_p,  alpha_p = delta_p + c_p,
// which only adds and multiplies positive numbers, so every pivot keeps the
// relative accuracy of its inputs (the Schur complements of I + lambda L stay
// of the form identity plus a graph Laplacian; this is the bookkeeping of
// Grassmann, Taksar and Heyman for such matrices).  Forward substitution
// z_p = f_p + (c_{p-1} / alpha_{p-1}) z_{p-1} and back substitution
// u_p = (z_p + c_p u_{p+1}) / alpha_p follow Eqs. (15)-(20).
//
// The mode solves every strip serially, one thread per strip, as the paper
// does: it is a precision reference for float32 arithmetic, not a fast path
// (the partitioned kernels do not use it).  Thread ki keeps its strip's
// elimination in a buffer of one 16-byte record per element (two for four
// channels): element p of strip ki at buf[(p * nK + ki) * NVP + v], v = 0
// the ratio c_p / alpha_p, v = 1.. the channels, so that each element costs
// one vector store forward and one load and one store back, and the threads
// of a wave touch consecutive records.  A second kernel averages the strips
// covering each pixel (Sec. 2.3).
#include "sgwls_device.hpp"

namespace sgwls {
namespace {

// Floats per element record of the strip buffer (NC channels + the ratio,
// padded to whole 16-byte words).
template <int NC>
constexpr int delta_record() { return NC + 1 <= 4 ? 4 : 8; }

// Values (guidance plus channels, or ratio plus channels) a thread loads per
// batch of snake elements: one batch is in flight while the previous one is
// eliminated, and a thread has a SIMD to itself (a pass has one thread per
// strip), so the batch is as large as the registers allow.
constexpr int kDeltaValues = 160;

// Pixel offset of snake element p of the strip centred at k (r = 1).
DEV long long delta_pixel(const PassGeom& geo, int k, int p) {
  const int a = p / 3, q = p - 3 * a;
  const int b = (a & 1) ? k + 1 - q : k - 1 + q;
  return (long long)a * geo.sa + (long long)b * geo.sb;
}

template <int NC, int KIND>
__global__ __launch_bounds__(kWave) void k_delta_solve(const float* __restrict__ X,
                                                       const float* __restrict__ G, int c0,
                                                       PassGeom geo, WeightParams wp,
                                                       const float* __restrict__ lam_dev,
                                                       float lam_host, float* __restrict__ buf) {
  const int ki = blockIdx.x * kWave + threadIdx.x;
  if (ki >= geo.nK) return;
  const int k = min(1 + ki * geo.stride, geo.W - 2);
  const float lamS = load_lambda(lam_dev, lam_host) * wp.spatial[1];
  const int s = 3 * geo.L;
  const size_t nK = geo.nK;
  constexpr int NV = NC + 1, D = kDeltaValues / NV, NVP = delta_record<NC>();
  const float* Xc = X + (size_t)c0 * geo.plane;
  auto rec = [&](int p) -> float4* {
    return reinterpret_cast<float4*>(buf + ((size_t)p * nK + ki) * NVP);
  };
  // record p <- (ratio, values[0..NC)), zero-padded
  auto put = [&](int p, float ratio, const float (&vals)[NC]) {
    float w[NVP] = {};
    w[0] = ratio;
#pragma unroll
    for (int h = 0; h < NC; ++h) w[1 + h] = vals[h];
    float4* d = rec(p);
#pragma unroll
    for (int q = 0; q < NVP / 4; ++q) d[q] = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  };
  auto get = [&](int p, float& ratio, float (&vals)[NC]) {
    float w[NVP];
    const float4* d = rec(p);
#pragma unroll
    for (int q = 0; q < NVP / 4; ++q) {
      const float4 t = d[q];
      w[4 * q] = t.x;
      w[4 * q + 1] = t.y;
      w[4 * q + 2] = t.z;
      w[4 * q + 3] = t.w;
    }
    ratio = w[0];
#pragma unroll
    for (int h = 0; h < NC; ++h) vals[h] = w[1 + h];
  };

  // Forward elimination, the loads of the next batch in flight meanwhile.
  // Loads past the end read the last element (clamped index, no branch) and
  // the arithmetic runs unconditionally, so that no load is sunk into a
  // per-element branch next to its use; only the stores are guarded.
  float gc[D], fc[D][NC], gn[D] = {}, fn[D][NC] = {};
  auto load = [&](int p0, float (&gg)[D], float (&ff)[D][NC]) {
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const long long o = delta_pixel(geo, k, min(p0 + e, s - 1));
      gg[e] = G[o];
#pragma unroll
      for (int h = 0; h < NC; ++h) ff[e][h] = Xc[(size_t)h * geo.plane + o];
    }
  };
  load(0, gc, fc);
  float delta = 1.0f, ratio_prev = 0.0f;
  float z[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) z[h] = 0.0f;
  for (int p0 = 0; p0 < s; p0 += D) {
    if (p0 + D < s) load(p0 + D, gn, fn);
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int p = p0 + e;
      const float gnext = e + 1 < D ? gc[e + 1 < D ? e + 1 : 0] : gn[0];   // next batch's first
      const float c = p + 1 < s ? lamS * range_weight<KIND>(gnext - gc[e], wp) : 0.0f;
      const float alpha = delta + c;
      const float inv = 1.0f / alpha;
      const float ratio = c * inv;
      float zs[NC];
#pragma unroll
      for (int h = 0; h < NC; ++h) {
        z[h] = fc[e][h] + ratio_prev * z[h];
        zs[h] = z[h] * inv;
      }
      if (p < s) put(p, ratio, zs);
      delta = 1.0f + c * (delta * inv);
      ratio_prev = ratio;
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      gc[e] = gn[e];
#pragma unroll
      for (int h = 0; h < NC; ++h) fc[e][h] = fn[e][h];
    }
  }

  // back substitution u_p = z_p / alpha_p + (c_p / alpha_p) u_{p+1}, in place
  float u[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) u[h] = 0.0f;
  const int nb = (s + D - 1) / D;
  float rc[D], zc[D][NC], rn[D] = {}, zn[D][NC] = {};
  auto load_back = [&](int b, float (&rr)[D], float (&zz)[D][NC]) {
#pragma unroll
    for (int e = 0; e < D; ++e) get(min(b * D + e, s - 1), rr[e], zz[e]);
  };
  load_back(nb - 1, rc, zc);
  for (int b = nb - 1; b >= 0; --b) {
    if (b > 0) load_back(b - 1, rn, zn);
#pragma unroll
    for (int e = D - 1; e >= 0; --e) {
      const int p = b * D + e;
      // elements past the end (the last batch's tail) leave u at 0
      const bool live = p < s;
#pragma unroll
      for (int h = 0; h < NC; ++h) u[h] = live ? zc[e][h] + rc[e] * u[h] : 0.0f;
      if (live) put(p, rc[e], u);
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      rc[e] = rn[e];
#pragma unroll
      for (int h = 0; h < NC; ++h) zc[e][h] = zn[e][h];
    }
  }
}

// Output pixel (a, b) of the pass: the mean over the strips whose centres
// lie within one column of b (Sec. 2.3), in increasing strip order.  With
// geo.out_t the output is stored transposed (pixel (a, b) at b * L + a),
// which is the layout the next pass reads as a column pass.
template <int NC>
__global__ __launch_bounds__(256) void k_delta_average(const float* __restrict__ buf,
                                                       float* __restrict__ Y, int c0,
                                                       PassGeom geo) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)geo.L * geo.W) return;
  const int a = (int)(idx / geo.W), b = (int)(idx - (long long)a * geo.W);
  const int t = geo.stride, last = geo.nK - 1;
  const size_t nK = geo.nK;
  constexpr int NVP = delta_record<NC>();
  float acc[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) acc[h] = 0.0f;
  int cnt = 0;
  auto add = [&](int ki) {
    const int k = min(1 + ki * t, geo.W - 2);
    if (k < b - 1 || k > b + 1) return;
    const int q = (a & 1) ? k + 1 - b : b - (k - 1);
    const int p = 3 * a + q;
#pragma unroll
    for (int h = 0; h < NC; ++h) acc[h] += buf[((size_t)p * nK + ki) * NVP + 1 + h];
    ++cnt;
  };
  // regular centres 1 + ki t in [b - 1, b + 1], then the appended last one
  const int lo = b - 2 <= 0 ? 0 : (b - 2 + t - 1) / t;
  const int hi = min(last, b / t);
  for (int ki = lo; ki <= hi; ++ki) add(ki);
  if (last > hi) add(last);
  const long long o = geo.out_t ? (long long)b * geo.L + a : (long long)a * geo.sa + (long long)b * geo.sb;
#pragma unroll
  for (int h = 0; h < NC; ++h) Y[(size_t)(c0 + h) * geo.plane + o] = acc[h] / (float)cnt;
}

template <int NC>
hipError_t delta_group(const float* x, const float* g, float* y, int c0, const PassGeom& geo,
                       const WeightParams& wp, const float* lam_dev, float lam_host, float* buf,
                       hipStream_t s) {
  const dim3 gs((geo.nK + kWave - 1) / kWave);
  if (wp.kind == 0)
    hipLaunchKernelGGL((k_delta_solve<NC, 0>), gs, dim3(kWave), 0, s, x, g, c0, geo, wp, lam_dev,
                       lam_host, buf);
  else
    hipLaunchKernelGGL((k_delta_solve<NC, 1>), gs, dim3(kWave), 0, s, x, g, c0, geo, wp, lam_dev,
                       lam_host, buf);
  const long long px = (long long)geo.L * geo.W;
  hipLaunchKernelGGL((k_delta_average<NC>), dim3((unsigned)((px + 255) / 256)), dim3(256), 0, s,
                     buf, y, c0, geo);
  return hipGetLastError();
}

}  // namespace

size_t delta_buffer_bytes(int C, int M, int N, int stride) {
  const size_t nv = std::min(C, kDeltaGroup) + 1 <= 4 ? 4 : 8;   // record floats (delta_record)
  const size_t col = (size_t)strip_count(N, 1, stride) * 3 * M;
  const size_t row = (size_t)strip_count(M, 1, stride) * 3 * N;
  return sizeof(float) * nv * std::max(col, row);
}

hipError_t launch_delta_pass(const float* x, const float* g, float* y, int C,
                             const PassGeom& geo, const WeightParams& wp, const float* lam_dev,
                             float lam_host, float* buf, hipStream_t s) {
  for (int c0 = 0; c0 < C; c0 += kDeltaGroup) {
    const int nc = std::min(kDeltaGroup, C - c0);
    hipError_t e;
    switch (nc) {
      case 1: e = delta_group<1>(x, g, y, c0, geo, wp, lam_dev, lam_host, buf, s); break;
      case 2: e = delta_group<2>(x, g, y, c0, geo, wp, lam_dev, lam_host, buf, s); break;
      case 3: e = delta_group<3>(x, g, y, c0, geo, wp, lam_dev, lam_host, buf, s); break;
      default: e = delta_group<4>(x, g, y, c0, geo, wp, lam_dev, lam_host, buf, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sgwls
