// Persistent kernels for batches of uneven images (every pass a direct-read
// column pass storing transposed, as for single images).  Each workgroup
// strides over the units of its stage (unit s, then s + gridDim.x, ..., with
// s its rank in the XCD-contiguous order, so that each XCD works on
// neighbouring units whose halos share its L2),
// locates each unit's image over the unit prefix sums and runs the same block
// code as the single-image kernels for that image's geometry and lambda.
// Units are ordered largest image first (the host sorts the table), so the
// tail of a launch is made of small blocks.  A static stride replaces a shared
// work counter: atomics on one address serialise at the L2 and cost more than
// the balance they buy across units of near-equal size.
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

// Image of unit u, remembered with its unit range [lo, hi): consecutive
// units of a workgroup mostly fall in one image (units are handed out in
// increasing order), which then costs no search.
struct Cursor {
  int i = 0, lo = 0, hi = 0;
  DEV int locate(const int* __restrict__ pre, int B, int u) {
    if (u < lo || u >= hi) {
      i = unit_image(pre, B, u);
      lo = pre[i];
      hi = pre[i + 1];
    }
    return i;
  }
};

// Every pass is a column pass storing its output transposed: pass 2t reads
// the image (f, then u) and writes tmp (N x M); pass 2t+1 reads tmp -- the
// row pass, on the transposed image -- and writes u.
DEV const float* pass_in(const BatchDesc& D, int q) {
  if (q == 0) return D.f;
  return (q % 2) ? D.tmp : D.u;
}
DEV float* pass_out(const BatchDesc& D, int q) { return (q % 2) ? D.u : D.tmp; }

// The kernels of one radius: a batch runs one launch per stage and radius
// over the images of that radius, so each kernel holds the registers of its
// own radius only.
template <int r, int CB, int KIND, typename Acc, int R, int Q>
__global__ __launch_bounds__(kWave* Q) void k_batch_reduce(const BatchDesc* __restrict__ tab,
                                                           const int* __restrict__ pre, int B,
                                                           int q, int dir,
                                                           Acc* __restrict__ iface) {
  extern __shared__ float smem[];
  const int total = pre[B];
  Cursor cur;
  const int slot = xcd_rank(blockIdx.x, gridDim.x);   // neighbouring units on one XCD
  for (int u = slot; u < total; u += gridDim.x) {
    __syncthreads();   // the previous unit is finished with the LDS
    const int i = cur.locate(pre, B, u);
    const BatchDesc& D = tab[i];
    int local = u - cur.lo;
    const int nbx = D.nbx_red[dir], per_c = nbx * D.nby[dir];
    const int c = local / per_c;   // channel block
    local -= c * per_c;
    const int by = local / nbx, bx = local - by * nbx;
    const PassGeom& geo = D.geo[dir];
    const PlaneSrc<CB> src{pass_in(D, q), nullptr, c * CB, (int)geo.plane};
    const float* gf = dir ? D.gT : D.g;
    Acc* sum = iface + D.sum_base + c * D.sum_ch;
    reduce_tile<r, CB, R, Q, true, KIND, Acc, kModeForward, true>(geo, D.wp, D.lam, 0, sum, bx,
                                                                  by, smem, gf, &src);
  }
}

// kIfaceWaves independent waves per workgroup, each solving the separator
// systems of its own (image, channel, strip) units (the solver is
// wave-local: no workgroup barrier).
constexpr int kIfaceWaves = 4;

template <int r, int CB, typename Acc>
__global__ __launch_bounds__(kWave* kIfaceWaves) void k_batch_iface(
    const BatchDesc* __restrict__ tab, const int* __restrict__ pre, int B, int dir,
    Acc* __restrict__ iface) {
  const int total = pre[B];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  Cursor cur;
  for (int u = blockIdx.x * kIfaceWaves + wave; u < total; u += gridDim.x * kIfaceWaves) {
    const int i = cur.locate(pre, B, u);
    const BatchDesc& D = tab[i];
    const int local = u - cur.lo;
    const int nK = D.geo[dir].nK;
    const int c = local / nK, ki = local - c * nK;   // channel block, strip
    const Acc* sum = iface + D.sum_base + c * D.sum_ch;
    Acc* us = iface + D.us_base + c * D.us_ch;
    iface_pcr_strip<r, CB, kBatchMM, Acc>(sum, us, D.geo[dir].P, D.m[dir], ki);
  }
}

template <int r, int CB, int KIND, typename Acc, int R, int Q>
__global__ __launch_bounds__(kWave* Q) void k_batch_expand(const BatchDesc* __restrict__ tab,
                                                           const int* __restrict__ pre, int B,
                                                           int q, int dir,
                                                           const Acc* __restrict__ iface) {
  extern __shared__ float smem[];
  const int total = pre[B];
  const BwdArgs none{};
  Cursor cur;
  const int slot = xcd_rank(blockIdx.x, gridDim.x);   // neighbouring units on one XCD
  for (int u = slot; u < total; u += gridDim.x) {
    __syncthreads();   // the previous unit is finished with the LDS
    const int i = cur.locate(pre, B, u);
    const BatchDesc& D = tab[i];
    int local = u - cur.lo;
    const int nbx = D.nbx_exp[dir], per_c = nbx * D.nby[dir];
    const int c = local / per_c;   // channel block
    local -= c * per_c;
    const int by = local / nbx, bx = local - by * nbx;
    const PassGeom& geo = D.geo[dir];
    const PlaneSrc<CB> src{pass_in(D, q), nullptr, c * CB, (int)geo.plane};
    const float* gf = dir ? D.gT : D.g;
    float* y = pass_out(D, q);
    const Acc* us = iface + D.us_base + c * D.us_ch;
    expand_tile<r, CB, R, Q, true, KIND, Acc, kModeForward, true>(gf, y, geo, D.wp, D.lam, c * CB,
                                                                  us, D.OW, 0, none, bx, by, nbx,
                                                                  smem, &src);
  }
}

// LDS of one batched reduce / expand block (direct reads: the reduce output
// staging and the transposed-store staging).
template <typename Acc, int r, int CB, int R, int Q>
constexpr size_t batch_lds() {
  const size_t out = sizeof(float) * CB * Q * R * (kWave + 1);
  const size_t F = r * (r + 1) + 2 * r * CB + r * r;
  const size_t stage = sizeof(Acc) * kWave * Q * F;
  return out > stage ? out : stage;
}

// Guidance transposes of a batch: one 32 x 32 tile per workgroup.
__global__ __launch_bounds__(256) void k_batch_transpose(const BatchDesc* __restrict__ tab,
                                                         const int* __restrict__ pre, int B) {
  __shared__ float t[32][33];
  const int u = blockIdx.x;
  const int i = unit_image(pre, B, u);
  const BatchDesc& D = tab[i];
  const int rows = D.M, cols = D.N;
  const int tiles_x = (cols + 31) / 32;
  const int local = u - pre[i];
  const int c0 = (local % tiles_x) * 32, r0 = (local / tiles_x) * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += 8) {
    const int rr = r0 + k, cc = c0 + tx;
    if (rr < rows && cc < cols) t[k][tx] = D.g[(size_t)rr * cols + cc];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int cc = c0 + k, rr = r0 + tx;
    if (rr < rows && cc < cols) D.gT[(size_t)cc * rows + rr] = t[tx][k];
  }
}

// Resident workgroups of a kernel over the whole device (the persistent
// grid), from its register and LDS footprint: 512 VGPRs per lane and at
// most 8 waves per SIMD, 4 SIMDs and 160 KiB of LDS per compute unit.
// Workgroups beyond what fits only start late and find the queue drained.
template <typename K>
int persistent_grid(K kernel, int block, size_t lds) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
  const int vgprs = std::max(8, (fa.numRegs + 7) / 8 * 8);
  const int waves_simd = std::min(8, 512 / vgprs);
  const int waves_wg = (block + kWave - 1) / kWave;
  int per_cu = std::max(1, waves_simd * 4 / waves_wg);
  const size_t lds_wg = lds + fa.sharedSizeBytes;
  if (lds_wg > 0) per_cu = std::min<long long>(per_cu, std::max<size_t>(1, (160u << 10) / lds_wg));
  return per_cu * std::max(1, cus);
}

template <int r, int CB, int KIND, typename Acc, int R, int Q>
hipError_t batch_pass_impl(const BatchDesc* tab, const int* pre_r, const int* pre_i,
                           const int* pre_e, const int totals[3], int B, int q, int dir,
                           void* iface, hipStream_t s) {
  Acc* buf = reinterpret_cast<Acc*>(iface);
  constexpr size_t lds = batch_lds<Acc, r, CB, R, Q>();
  static const int g_red =
      persistent_grid(k_batch_reduce<r, CB, KIND, Acc, R, Q>, kWave * Q, lds);
  static const int g_if = persistent_grid(k_batch_iface<r, CB, Acc>, kWave * kIfaceWaves, 0);
  static const int g_exp =
      persistent_grid(k_batch_expand<r, CB, KIND, Acc, R, Q>, kWave * Q, lds);
  if (g_red <= 0 || g_if <= 0 || g_exp <= 0) return hipErrorInvalidConfiguration;
  if (totals[0] + totals[1] + totals[2] == 0) return hipSuccess;
  if (totals[0] > 0)
    hipLaunchKernelGGL((k_batch_reduce<r, CB, KIND, Acc, R, Q>), dim3(std::min(g_red, totals[0])),
                       dim3(kWave * Q), lds, s, tab, pre_r, B, q, dir, buf);
  if (totals[1] > 0)
    hipLaunchKernelGGL((k_batch_iface<r, CB, Acc>),
                       dim3(std::min(g_if, (totals[1] + kIfaceWaves - 1) / kIfaceWaves)),
                       dim3(kWave * kIfaceWaves), 0, s, tab, pre_i, B, dir, buf);
  if (totals[2] > 0)
    hipLaunchKernelGGL((k_batch_expand<r, CB, KIND, Acc, R, Q>), dim3(std::min(g_exp, totals[2])),
                       dim3(kWave * Q), lds, s, tab, pre_e, B, q, dir, (const Acc*)buf);
  return hipGetLastError();
}

template <int KIND, int fp64, int V>
hipError_t batch_variant_impl(int v, int r, const BatchDesc* tab, const int* pre_r,
                              const int* pre_i, const int* pre_e, const int totals[3], int B,
                              int q, int dir, void* iface, hipStream_t s) {
  if constexpr (V < batch_variant_count(fp64)) {
    if (v == V) {
      constexpr BatchVariant bv = batch_variant(V, fp64);
      using Acc = typename std::conditional<fp64 != 0, double, float>::type;
      if (r == 1)
        return batch_pass_impl<1, 1, KIND, Acc, bv.R1, bv.Q>(tab, pre_r, pre_i, pre_e, totals, B,
                                                             q, dir, iface, s);
      if (r == 2)
        return batch_pass_impl<2, 1, KIND, Acc, bv.R2, bv.Q>(tab, pre_r, pre_i, pre_e, totals, B,
                                                             q, dir, iface, s);
      return hipErrorInvalidValue;
    }
    return batch_variant_impl<KIND, fp64, V + 1>(v, r, tab, pre_r, pre_i, pre_e, totals, B, q,
                                                 dir, iface, s);
  } else {
    return hipErrorInvalidValue;
  }
}

// Three-channel blocks: the chunk shape of the single-image path's first
// (direct) variant for three channels.
template <int KIND, int fp64>
hipError_t batch_cb3_impl(int r, const BatchDesc* tab, const int* pre_r, const int* pre_i,
                          const int* pre_e, const int totals[3], int B, int q, int dir,
                          void* iface, hipStream_t s) {
  using Acc = typename std::conditional<fp64 != 0, double, float>::type;
  constexpr VariantSet v1 = variants_of(1, 3, fp64), v2 = variants_of(2, 3, fp64);
  if (r == 1)
    return batch_pass_impl<1, 3, KIND, Acc, v1.v[0].R, v1.v[0].Q>(tab, pre_r, pre_i, pre_e,
                                                                  totals, B, q, dir, iface, s);
  if (r == 2)
    return batch_pass_impl<2, 3, KIND, Acc, v2.v[0].R, v2.v[0].Q>(tab, pre_r, pre_i, pre_e,
                                                                  totals, B, q, dir, iface, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_pass(int variant, int fp64, int kind, int r, int cb, const BatchDesc* tab,
                             const int* pre_r, const int* pre_i, const int* pre_e,
                             const int totals[3], int B, int q, int dir, void* iface,
                             hipStream_t s) {
  if (cb == 3) {
    if (kind == 0)
      return fp64 ? batch_cb3_impl<0, 1>(r, tab, pre_r, pre_i, pre_e, totals, B, q, dir, iface, s)
                  : batch_cb3_impl<0, 0>(r, tab, pre_r, pre_i, pre_e, totals, B, q, dir, iface, s);
    return fp64 ? batch_cb3_impl<1, 1>(r, tab, pre_r, pre_i, pre_e, totals, B, q, dir, iface, s)
                : batch_cb3_impl<1, 0>(r, tab, pre_r, pre_i, pre_e, totals, B, q, dir, iface, s);
  }
  if (kind == 0)
    return fp64 ? batch_variant_impl<0, 1, 0>(variant, r, tab, pre_r, pre_i, pre_e, totals, B, q,
                                              dir, iface, s)
                : batch_variant_impl<0, 0, 0>(variant, r, tab, pre_r, pre_i, pre_e, totals, B, q,
                                              dir, iface, s);
  return fp64 ? batch_variant_impl<1, 1, 0>(variant, r, tab, pre_r, pre_i, pre_e, totals, B, q,
                                            dir, iface, s)
              : batch_variant_impl<1, 0, 0>(variant, r, tab, pre_r, pre_i, pre_e, totals, B, q,
                                            dir, iface, s);
}

hipError_t launch_batch_transpose(const BatchDesc* tab, const int* pre_t, int B, int tiles,
                                  hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_transpose, dim3(tiles), dim3(256), 0, s, tab, pre_t, B);
  return hipGetLastError();
}

}  // namespace sgwls
