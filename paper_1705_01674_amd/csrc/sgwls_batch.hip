// Persistent kernels for batches of uneven images.  Each workgroup loops:
// take the next unit from the stage's counter, locate its image by binary
// search over the unit prefix sums, run the same block code as the
// single-image kernels for that image's geometry, radius and lambda.  Units
// are ordered largest image first (the host sorts the table), so the tail of
// a launch is made of small blocks.
#include "sgwls_device.hpp"

namespace sgwls {
namespace {

// Last image whose first unit is <= u (images without units are skipped
// because their prefix equals the next one's).
DEV int unit_image(const int* __restrict__ pre, int B, int u) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Input and output of pass q (x_0 = f, x_passes = u; the others alternate
// between tmp and u so that the last pass lands in u).
DEV const float* pass_in(const BatchDesc& D, int q, int passes) {
  if (q == 0) return D.f;
  return ((passes - (q - 1)) % 2 == 0) ? D.tmp : D.u;
}
DEV float* pass_out(const BatchDesc& D, int q, int passes) {
  if (q == passes - 1) return D.u;
  return ((passes - q) % 2 == 0) ? D.tmp : D.u;
}

// Next unit of the workgroup (all threads receive the same value).
DEV int next_unit(int* counter, int* slot) {
  __syncthreads();   // the previous unit is finished with the LDS and the slot
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*slot);
}

template <int KIND, typename Acc, int R1, int R2, int Q>
__global__ __launch_bounds__(kWave* Q) void k_batch_reduce(const BatchDesc* __restrict__ tab,
                                                           const int* __restrict__ pre, int B,
                                                           int q, int passes, int dir,
                                                           int* counter, Acc* __restrict__ iface) {
  extern __shared__ float smem[];
  __shared__ int slot;
  const int total = pre[B];
  for (;;) {
    const int u = next_unit(counter, &slot);
    if (u >= total) break;
    const int i = unit_image(pre, B, u);
    const BatchDesc& D = tab[i];
    int local = u - pre[i];
    const int nbx = D.nbx_red[dir], per_c = nbx * D.nby[dir];
    const int c = local / per_c;
    local -= c * per_c;
    const int by = local / nbx, bx = local - by * nbx;
    const float* x = pass_in(D, q, passes);
    Acc* sum = iface + D.sum_base + c * D.sum_ch;
    if (D.r == 1)
      reduce_block<1, 1, R1, Q, true, KIND, Acc, kModeForward>(x, nullptr, D.g, D.geo[dir], D.wp,
                                                               D.lam, c, 0, sum, bx, by, smem);
    else
      reduce_block<2, 1, R2, Q, true, KIND, Acc, kModeForward>(x, nullptr, D.g, D.geo[dir], D.wp,
                                                               D.lam, c, 0, sum, bx, by, smem);
  }
}

// One wave per workgroup; each wave solves the separator system of one
// (image, channel, strip) unit at a time.
template <typename Acc>
__global__ __launch_bounds__(kWave) void k_batch_iface(const BatchDesc* __restrict__ tab,
                                                       const int* __restrict__ pre, int B,
                                                       int dir, int* counter,
                                                       Acc* __restrict__ iface) {
  __shared__ int slot;
  const int total = pre[B];
  for (;;) {
    const int u = next_unit(counter, &slot);
    if (u >= total) break;
    const int i = unit_image(pre, B, u);
    const BatchDesc& D = tab[i];
    const int local = u - pre[i];
    const int nK = D.geo[dir].nK;
    const int c = local / nK, ki = local - c * nK;
    const Acc* sum = iface + D.sum_base + c * D.sum_ch;
    Acc* us = iface + D.us_base + c * D.us_ch;
    if (D.r == 1)
      iface_pcr_strip<1, 1, kBatchMM, Acc>(sum, us, D.geo[dir].P, D.m[dir], ki);
    else
      iface_pcr_strip<2, 1, kBatchMM, Acc>(sum, us, D.geo[dir].P, D.m[dir], ki);
  }
}

template <int KIND, typename Acc, int R1, int R2, int Q>
__global__ __launch_bounds__(kWave* Q) void k_batch_expand(const BatchDesc* __restrict__ tab,
                                                           const int* __restrict__ pre, int B,
                                                           int q, int passes, int dir,
                                                           int* counter,
                                                           const Acc* __restrict__ iface) {
  extern __shared__ float smem[];
  __shared__ int slot;
  const int total = pre[B];
  const BwdArgs none{};
  for (;;) {
    const int u = next_unit(counter, &slot);
    if (u >= total) break;
    const int i = unit_image(pre, B, u);
    const BatchDesc& D = tab[i];
    int local = u - pre[i];
    const int nbx = D.nbx_exp[dir], per_c = nbx * D.nby[dir];
    const int c = local / per_c;
    local -= c * per_c;
    const int by = local / nbx, bx = local - by * nbx;
    const float* x = pass_in(D, q, passes);
    float* y = pass_out(D, q, passes);
    const Acc* us = iface + D.us_base + c * D.us_ch;
    if (D.r == 1)
      expand_block<1, 1, R1, Q, true, KIND, Acc, kModeForward>(x, D.g, y, D.geo[dir], D.wp, D.lam,
                                                               c, us, D.OW, 0, none, bx, by, nbx,
                                                               smem);
    else
      expand_block<2, 1, R2, Q, true, KIND, Acc, kModeForward>(x, D.g, y, D.geo[dir], D.wp, D.lam,
                                                               c, us, D.OW, 0, none, bx, by, nbx,
                                                               smem);
  }
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// LDS of one batched reduce / expand block: the larger radius decides.
template <typename Acc, int R1, int R2, int Q>
size_t batch_lds() {
  size_t need = 0;
  const int R[2] = {R1, R2};
  for (int r = 1; r <= kBatchMaxR; ++r) {
    const size_t pitch = kWave + 2 * r + 1;
    const size_t tile = sizeof(float) * 2 * (Q * R[r - 1] + 2) * pitch;
    const size_t F = r * (r + 1) + 2 * r + r * r;
    const size_t stage = sizeof(Acc) * kWave * Q * F;
    need = std::max(need, std::max(tile, stage));
  }
  return need;
}

// Resident workgroups of a kernel over the whole device (the persistent grid).
template <typename K>
int persistent_grid(K kernel, int block, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess)
    return 0;
  return std::max(1, per_cu) * std::max(1, cus);
}

template <int KIND, typename Acc, int R1, int R2, int Q>
hipError_t batch_pass_impl(const BatchDesc* tab, const int* pre_r, const int* pre_i,
                           const int* pre_e, const int totals[3], int B, int q, int passes,
                           int dir, int* counters, void* iface, hipStream_t s) {
  Acc* buf = reinterpret_cast<Acc*>(iface);
  const size_t lds = batch_lds<Acc, R1, R2, Q>();
  static const int g_red = persistent_grid(k_batch_reduce<KIND, Acc, R1, R2, Q>, kWave * Q, lds);
  static const int g_if = persistent_grid(k_batch_iface<Acc>, kWave, 0);
  static const int g_exp = persistent_grid(k_batch_expand<KIND, Acc, R1, R2, Q>, kWave * Q, lds);
  if (g_red <= 0 || g_if <= 0 || g_exp <= 0) return hipErrorInvalidConfiguration;
  if (totals[0] + totals[1] + totals[2] == 0) return hipSuccess;
  if (totals[0] > 0)
    hipLaunchKernelGGL((k_batch_reduce<KIND, Acc, R1, R2, Q>), dim3(std::min(g_red, totals[0])),
                       dim3(kWave * Q), lds, s, tab, pre_r, B, q, passes, dir, counters + 0, buf);
  if (totals[1] > 0)
    hipLaunchKernelGGL((k_batch_iface<Acc>), dim3(std::min(g_if, totals[1])), dim3(kWave), 0, s,
                       tab, pre_i, B, dir, counters + 1, buf);
  if (totals[2] > 0)
    hipLaunchKernelGGL((k_batch_expand<KIND, Acc, R1, R2, Q>), dim3(std::min(g_exp, totals[2])),
                       dim3(kWave * Q), lds, s, tab, pre_e, B, q, passes, dir, counters + 2,
                       (const Acc*)buf);
  return hipGetLastError();
}

template <int KIND, int fp64, int V>
hipError_t batch_variant_impl(int v, const BatchDesc* tab, const int* pre_r, const int* pre_i,
                              const int* pre_e, const int totals[3], int B, int q, int passes,
                              int dir, int* counters, void* iface, hipStream_t s) {
  if constexpr (V < batch_variant_count(fp64)) {
    if (v == V) {
      constexpr BatchVariant bv = batch_variant(V, fp64);
      using Acc = typename std::conditional<fp64 != 0, double, float>::type;
      return batch_pass_impl<KIND, Acc, bv.R1, bv.R2, bv.Q>(tab, pre_r, pre_i, pre_e, totals, B,
                                                            q, passes, dir, counters, iface, s);
    }
    return batch_variant_impl<KIND, fp64, V + 1>(v, tab, pre_r, pre_i, pre_e, totals, B, q,
                                                 passes, dir, counters, iface, s);
  } else {
    return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_batch_pass(int variant, int fp64, int kind, const BatchDesc* tab,
                             const int* pre_r, const int* pre_i, const int* pre_e,
                             const int totals[3], int B, int q, int passes, int dir,
                             int* counters, void* iface, hipStream_t s) {
  if (kind == 0)
    return fp64 ? batch_variant_impl<0, 1, 0>(variant, tab, pre_r, pre_i, pre_e, totals, B, q,
                                              passes, dir, counters, iface, s)
                : batch_variant_impl<0, 0, 0>(variant, tab, pre_r, pre_i, pre_e, totals, B, q,
                                              passes, dir, counters, iface, s);
  return fp64 ? batch_variant_impl<1, 1, 0>(variant, tab, pre_r, pre_i, pre_e, totals, B, q,
                                            passes, dir, counters, iface, s)
              : batch_variant_impl<1, 0, 0>(variant, tab, pre_r, pre_i, pre_e, totals, B, q,
                                            passes, dir, counters, iface, s);
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace sgwls
