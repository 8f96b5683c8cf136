// Radius-independent kernels: the fix-up step of a backward pass and small
// stream-ordered writes of host data.
#include "sgwls_internal.hpp"

namespace sgwls {
namespace {

constexpr int kFixThreads = 256;

// Blocks [0, nfix): side terms of chunk j (guidance-gradient terms of edges
// from chunk j-1's last r elements into chunk j, gathered per pixel by the
// expand kernel) are added to the pixels of row jR - 1.  Block nfix (when
// lpart is set): fixed-order reduction of the per-block lambda partials.
__global__ __launch_bounds__(kFixThreads) void k_bwd_fixup(const float* __restrict__ side,
                                                           float* __restrict__ gbar,
                                                           PassGeom geo, int nfix,
                                                           const double* __restrict__ lpart,
                                                           int nparts, double* glam,
                                                           int lam_acc) {
  // blockIdx.z: image of a batched launch (side terms per image; the lambda
  // partials of every image are reduced together by block (nfix, 0, 0))
  if ((int)blockIdx.x < nfix) {
    side = zmove(side, geo.zside, (int)blockIdx.z);
    gbar = zmove(gbar, geo.zgb, (int)blockIdx.z);
    const int idx = blockIdx.x * kFixThreads + threadIdx.x;
    const int n = (geo.P - 1) * geo.W;
    if (idx < n) {
      const int j = 1 + idx / geo.W, b = idx - (j - 1) * geo.W;
      const int a = j * geo.R - 1;
      const long long o = a * geo.sa + b * geo.sb;
      gbar[o] += side[(size_t)j * geo.W + b];
    }
    return;
  }
  if (blockIdx.z != 0) return;
  __shared__ double red[kFixThreads];
  // Each thread sums partials threadIdx.x, + kFixThreads, ... in that order;
  // kLoads of them are loaded before they are added, so that one memory
  // latency covers the batch.
  constexpr int kLoads = 16;
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < nparts; i0 += kFixThreads * kLoads) {
    double v[kLoads];
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int i = i0 + u * kFixThreads;
      v[u] = i < nparts ? lpart[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLoads; ++u) s += v[u];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kFixThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *glam = lam_acc ? *glam + red[0] : red[0];
}

__global__ __launch_bounds__(256) void k_write_words(unsigned int* __restrict__ dst, WordChunk c) {
  for (unsigned int i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

// 32 x 32 tiles through LDS (padded row), coalesced reads and writes.
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src,
                                                   float* __restrict__ dst, int rows, int cols,
                                                   int accumulate, unsigned int* zero,
                                                   int nzero) {
  __shared__ float t[32][33];
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0)
    for (int i = threadIdx.x; i < nzero; i += 256) zero[i] = 0u;
  const size_t plane = (size_t)rows * cols;
  src += blockIdx.z * plane;
  dst += blockIdx.z * plane;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int i = ty; i < 32; i += 8) {
    const int rr = r0 + i, cc = c0 + tx;
    if (rr < rows && cc < cols) t[i][tx] = src[(size_t)rr * cols + cc];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int cc = c0 + i, rr = r0 + tx;
    if (rr < rows && cc < cols) {
      float* d = dst + (size_t)cc * rows + rr;
      *d = accumulate ? *d + t[tx][i] : t[tx][i];
    }
  }
}

}  // namespace

hipError_t launch_transpose(const float* src, float* dst, int rows, int cols, hipStream_t stream,
                            int planes, int accumulate, unsigned int* zero, int nzero) {
  hipLaunchKernelGGL(k_transpose, dim3((cols + 31) / 32, (rows + 31) / 32, planes), dim3(256), 0,
                     stream, src, dst, rows, cols, accumulate, zero, nzero);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_words(unsigned int* __restrict__ dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = 0u;
}

hipError_t launch_zero_words(unsigned int* dst, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, stream, dst, n);
  return hipGetLastError();
}

hipError_t launch_write_words(unsigned int* dst, const WordChunk& c, hipStream_t stream) {
  if (c.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_write_words, dim3(1), dim3(256), 0, stream, dst, c);
  return hipGetLastError();
}

hipError_t launch_bwd_fixup(const float* side, float* gbar, const PassGeom& geo,
                            const double* lpart, int nparts, double* glam, int lam_acc,
                            hipStream_t stream) {
  const int nfix = gbar && geo.P > 1 ? ((geo.P - 1) * geo.W + kFixThreads - 1) / kFixThreads : 0;
  const int nlam = (lpart && glam) ? 1 : 0;
  if (nfix + nlam == 0) return hipSuccess;
  const int nz = geo.nimg > 0 ? geo.nimg : 1;
  hipLaunchKernelGGL(k_bwd_fixup, dim3(nfix + nlam, 1, nz), dim3(kFixThreads), 0, stream, side,
                     gbar, geo, nfix, lpart, nparts * nz, glam, lam_acc);
  return hipGetLastError();
}

// u[c] = num[c] / den for the C numerator planes (Eq. 21's quotient).
__global__ __launch_bounds__(256) void k_divide_planes(const float* __restrict__ num,
                                                       const float* __restrict__ den,
                                                       float* __restrict__ u, int C,
                                                       long long plane) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= plane) return;
  const float d = den[i];
  for (int c = 0; c < C; ++c) u[c * plane + i] = num[c * plane + i] / d;
}

hipError_t launch_divide_planes(const float* num, const float* den, float* u, int C,
                                long long plane, hipStream_t s) {
  if (plane <= 0 || C <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_divide_planes, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, num,
                     den, u, C, plane);
  return hipGetLastError();
}

}  // namespace sgwls
