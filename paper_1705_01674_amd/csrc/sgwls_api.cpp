// C ABI of the SG-WLS library (declared in include/sgwls.h).
//
// Host-side validation, workspace layout and the order of passes of Sec. 2.3
// (T iterations of a column pass followed by a row pass).  All device memory
// is supplied by the caller; nothing here allocates.
#include "sgwls.h"
#include "sgwls_internal.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

using namespace sgwls;

namespace {
sgwls_status validate_partitioned(int C, int M, int N, const sgwls_params* p);

constexpr int kVersion = 201;          // 0.2.1
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
// Strided passes are tuned apart from stride-1 ones: their direction field
// is offset by kStridedDir.
constexpr int kStridedDir = 4;
TuneKey tune_key(int r, int cb, int fp64, int kind, int dir, int L, int W) {
  return TuneKey(r, cb, fp64, kind, dir, size_bucket(L, W));
}
void tune_cache_load_once();
int tuned_variant(int r, int cb, int fp64, int kind, int dir, int L, int W) {
  tune_cache_load_once();
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

// Bound on the largest diagonal entry of A_s (Eq. 4 with the weights of
// Eq. 2): every element has at most two edges at each distance d = 1..r, each
// weighing at most S(d) times the largest range factor (1 for omega^exp,
// 1 / eps for omega^frac at equal guidance).
double auto_kappa(const sgwls_params& p) {
  double s = 0.0;
  for (int d = 1; d <= p.r; ++d)
    s += p.kind == SGWLS_W_EXP ? std::exp(-(double)d * d / (2.0 * (double)p.sigma_s * p.sigma_s))
                               : 1.0 / (std::pow((double)d, (double)p.alpha_s) + (double)p.eps);
  const double rmax = p.kind == SGWLS_W_EXP ? 1.0 : 1.0 / (double)p.eps;
  return 1.0 + 2.0 * (double)p.lambda * s * rmax;
}

// The parameters a call runs with: SGWLS_P_AUTO replaced by the precision it
// resolves to (see sgwls_precision in sgwls.h).
sgwls_params resolved(const sgwls_params& p, int want_lambda_grad) {
  sgwls_params q = p;
  if (p.prec == SGWLS_P_AUTO)
    q.prec = (want_lambda_grad || auto_kappa(p) > SGWLS_AUTO_KAPPA_MAX) ? SGWLS_P_FP64_PIVOT
                                                                       : SGWLS_P_FP32;
  return q;
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

// Fused forward passes (stage-ordered units with counter waits) in place of
// the three stage kernels, read at every call from SGWLS_ONE_LAUNCH: unset
// or 0 = three launches per pass, 1 = one launch, 2 = reduce and interface
// in one launch, expand in a second.
thread_local int t_no_fused = 0;
int one_launch_mode() {
  if (t_no_fused > 0) return 0;
  const char* e = std::getenv("SGWLS_ONE_LAUNCH");
  return (e && (e[0] == '1' || e[0] == '2')) ? e[0] - '0' : 0;
}
// Polls of one counter wait before it gives up: about two seconds, or
// SGWLS_FUSED_SPIN_LIMIT (a test of the error path sets it small).
unsigned int one_launch_spin_limit() {
  const char* e = std::getenv("SGWLS_FUSED_SPIN_LIMIT");
  if (e && e[0]) return (unsigned int)std::strtoul(e, nullptr, 10);
  return 1u << 20;
}

// Launch errors are read with hipGetLastError, which also returns an error
// left by an earlier, unrelated runtime call of the thread: clear it first.
void clear_hip_error() { (void)hipGetLastError(); }

// ---------------------------------------------------------------------------
// Saved separators.  The backward's recomputation of a pass needs the pass
// solution at the separators of the backward's chunks (variant 0 of the
// backward table); a filter call that keeps them lets every backward pass
// eliminate and solve only the adjoint system (one right-hand side per
// channel instead of two).  Where a forward variant is cut like the backward,
// the forward runs it and its interface writes its separator solutions
// straight to the buffer; otherwise the forward keeps its own chunks and its
// re-solve stores the last r elements of every subsystem row that ends a
// backward chunk (slower per pass: the stores sit in the re-solve).  The
// forward's transposed guidance goes to the buffer too, so that the backward
// need not transpose g again.  Buffer layout: the B transposed guidance
// planes (N x M each) rounded up to 256 bytes, then per image: pass q in
// order, then its channel blocks in order, each block the separator solutions
// in the backward's interface layout (r x cb values per separator, strip
// after strip) rounded up to 256 bytes.

// The backward's cut of a pass over an L x W frame (one channel block), with
// one right-hand side per channel: the layout of its separator solutions.
PassPlan seps_plan(int L, int W, int cb, const sgwls_params& p) {
  return make_plan(L, W, p.r, cb, 1, p.prec, 0, kModeAdjoint);
}

// Pass q of a stride-1 filter call runs as a column pass of an L x W frame:
// the image for even q, its transpose for odd q.
size_t seps_pass_bytes(int q, int C, int M, int N, const sgwls_params& p) {
  const int L = q % 2 == 0 ? M : N, W = q % 2 == 0 ? N : M;
  size_t b = 0;
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    const PassPlan pl = seps_plan(L, W, cb, p);
    b += align_up(pl.u_elems * pl.acc_bytes);
    c0 += cb;
  }
  return b;
}

// Bytes of the transposed guidance planes at the start of the buffer.
size_t seps_guidance_bytes(int B, int M, int N) {
  return align_up(sizeof(float) * (size_t)B * M * N);
}

// Per-image bytes of the separator regions, 0 when the case has no saved-
// separator path (p resolved, validated): stride-1 frames with direct
// forward and backward kernels, the partitioned precisions.
size_t seps_image_bytes(int C, int M, int N, const sgwls_params& p) {
  if (p.stride != 1 || (p.prec != SGWLS_P_FP32 && p.prec != SGWLS_P_FP64_PIVOT)) return 0;
  if (!frames_supported(C, p.r, 1, p.prec)) return 0;
  size_t b = 0;
  for (int q = 0; q < 2 * p.iters; ++q) b += seps_pass_bytes(q, C, M, N, p);
  return b;
}

// The whole buffer for B images, 0 when the case has no such path.
size_t seps_total_bytes(int B, int C, int M, int N, const sgwls_params& p) {
  const size_t per = seps_image_bytes(C, M, N, p);
  return per ? seps_guidance_bytes(B, M, N) + (size_t)B * per : 0;
}

// variant < 0: the tuned variant of the case (variant 0 when none is tuned).
sgwls_status enqueue_pass(int direction, const float* x, const float* g, float* y, int C, int M,
                          int N, const sgwls_params& p, const float* lam_dev, void* iface,
                          hipStream_t stream, int stages = kStageAll, int variant = -1,
                          const Batch* bt = nullptr, OneCtl* one = nullptr,
                          char* useps = nullptr, long long zseps = 0,
                          float* gT_out = nullptr) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const WeightParams wp = weight_params(p);
  const int out_t = (stages & kStageTransposeOut) ? 1 : 0;
  for (int c0 = 0; c0 < C;) {
    const int cb = channel_block(C - c0);
    int v = variant >= 0 ? variant
                         : tuned_variant(p.r, cb, p.prec, (int)p.kind,
                                         direction + (p.stride != 1 ? kStridedDir : 0), L, W);
    if (out_t && p.stride == 1 && !variants_of(p.r, cb, p.prec).v[v].D)
      v = 0;   // variant 0 reads directly
    const int sv = useps ? forward_variant_cut_like_backward(p.r, cb, p.prec) : -1;
    if (sv >= 0) v = sv;   // cut like the backward
    PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec, v);
    pl.one = useps ? nullptr : one;
    PassGeom geo = pass_geom(direction, M, N, pl, p.stride);
    geo.out_t = out_t;
    if (bt) set_batch(geo, *bt);
    BwdArgs keep{};
    if (useps) {
      const PassPlan sp = seps_plan(L, W, cb, p);
      if (sv >= 0) {
        // the interface writes its separator solutions to the buffer
        pl.us_out = useps;
        geo.zu = zseps;
      } else {
        // the re-solve stores the solution at the backward's separators
        keep.seps_out = useps;
        keep.zseps = zseps;
        keep.seps_R = sp.R;
        keep.seps_n = sp.P - 1;
      }
      useps += align_up(sp.u_elems * sp.acc_bytes);
    }
    if (gT_out && c0 == 0) {
      // the first block's re-solve transposes g when its staged tile, one
      // plane larger, still fits 64 KiB of LDS; else a transpose of its own
      const size_t lds = sizeof(float) * (size_t)(cb + 1) * pl.Q * pl.R * (kWave + 1);
      if (lds <= 65536)
        keep.gT_out = gT_out;
      else if (launch_transpose(g, gT_out, M, N, stream, bt ? bt->n : 1) != hipSuccess)
        return SGWLS_E_HIP;
    }
    stages &= kStageAll;
    hipError_t e = launch_pass(p.r, cb, p.prec, x, g, y, c0, geo, pl, wp, lam_dev, p.lambda,
                               iface, stream, stages,
                               (keep.seps_out || keep.gT_out) ? &keep : nullptr);
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
  size_t side_set, lpart_set;         // floats / doubles of one side / partials set
  size_t gt_off, gtacc_off, yt_off;   // transposed-frame buffers (frames only)
  size_t iface_img, side_img;         // per-image strides: bytes, floats
};

// B images (an NCHW batch): every buffer holds B per-image parts.
BwdLayout bwd_layout(int C, int M, int N, const sgwls_params& p, int B = 1) {
  size_t iface = 0, side = 0, blocks = 0;
  int nblk = 0;   // channel blocks
  for (int c0 = 0; c0 < C; c0 += channel_block(C - c0)) ++nblk;
  for (int dir = 0; dir < 2; ++dir) {
    const int L = dir == 0 ? M : N, W = dir == 0 ? N : M;
    for (int c0 = 0; c0 < C;) {
      const int cb = channel_block(C - c0);
      iface = std::max(iface, interface_bytes_max(L, W, p.r, cb, p.stride, p.prec, kModeBackward));
      if (p.stride == 1)   // the adjoint's own buffers (saved separators)
        iface = std::max(iface, interface_bytes(make_plan(L, W, p.r, cb, 1, p.prec, 0,
                                                          kModeAdjoint)));
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
  const size_t nb = (size_t)B;
  l.iface_img = align_up(iface);
  l.side_img = align_up(side * sizeof(float)) / sizeof(float);
  l.img_off = 0;
  l.iface_off = l.img_off + align_up(nb * sizeof(float) * C * M * N);
  // Side terms: one set per (frame parity, channel block); lambda partials:
  // one set per (pass, channel block).  A backward call over all passes
  // accumulates each set and applies them once at the end (set 0 alone when
  // every pass is fixed up by itself).
  l.side_set = nb * l.side_img;
  l.lpart_set = nb * blocks;
  const size_t nsides = 2 * (size_t)nblk, nparts = 2 * (size_t)p.iters * nblk;
  l.side_off = l.iface_off + nb * l.iface_img;
  l.lpart_off = l.side_off + align_up(nsides * l.side_set * sizeof(float));
  l.gt_off = l.lpart_off + align_up(nparts * l.lpart_set * sizeof(double));
  l.gtacc_off = l.gt_off + align_up(nb * sizeof(float) * M * N);
  l.yt_off = l.gtacc_off + align_up(nb * sizeof(float) * M * N);
  l.total = l.yt_off + align_up(nb * sizeof(float) * C * M * N);
  return l;
}

// Fix-ups deferred to the end of a backward call: the side terms of pass q,
// channel block b go to set side_set + b (added to the set when side_first
// is false), its lambda partials to the partials from lpart_off on.
struct BwdDefer {
  int side_set;
  bool side_first;
  size_t lpart_off;   // doubles from the start of the partials region
};

// One backward pass over all channel blocks.  `first` is true for the first
// launch of a backward call: it overwrites gbar and *grad_lambda, later
// launches add to them.  With dfr the fix-ups are left to the caller.
sgwls_status enqueue_pass_backward(int direction, const float* x, const float* g,
                                   const float* ybar, float* xbar, float* gbar,
                                   double* grad_lambda, int C, int M, int N,
                                   const sgwls_params& p, const float* lam_dev, void* ws,
                                   const BwdLayout& lay, hipStream_t stream, bool& first,
                                   bool* gfirst = nullptr, int out_t = 0,
                                   const Batch* bt = nullptr, const char* useps = nullptr,
                                   long long zseps = 0, BwdDefer* dfr = nullptr) {
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const WeightParams wp = weight_params(p);
  char* base = reinterpret_cast<char*>(ws);
  BwdArgs bw{};
  bw.ybar = ybar;
  bw.gbar = gbar;
  float* const side0 = reinterpret_cast<float*>(base + lay.side_off);
  double* const lpart0 = reinterpret_cast<double*>(base + lay.lpart_off);
  bw.side = side0;
  bw.lpart = grad_lambda ? lpart0 : nullptr;
  for (int c0 = 0, blk = 0; c0 < C; ++blk) {
    const int cb = channel_block(C - c0);
    PassPlan pl = make_plan(L, W, p.r, cb, p.stride, p.prec, 0, kModeBackward);
    PassGeom geo = pass_geom(direction, M, N, pl, p.stride);
    geo.out_t = out_t;
    if (bt) {
      // per image: its interface buffers, side terms and lambda partials (the
      // fix-up reduces the partials of every image together, in order)
      Batch b = *bt;
      b.iface = (long long)lay.iface_img;
      b.side = (long long)lay.side_img;
      b.lpart = expand_blocks(geo, pl);
      set_batch(geo, b);
    }
    bool& gf = gfirst ? *gfirst : first;   // first write of this guidance-gradient buffer
    bw.gacc = gf ? 0 : 1;
    if (dfr) {
      bw.side = side0 + (size_t)(dfr->side_set + blk) * lay.side_set;
      bw.sacc = dfr->side_first ? 0 : 1;
      bw.lpart = grad_lambda ? lpart0 + dfr->lpart_off : nullptr;
      dfr->lpart_off += (size_t)(bt ? bt->n : 1) * expand_blocks(geo, pl);
    }
    char* iface = base + lay.iface_off;
    int stages = kStageAll;
    if (useps) {
      // The pass solution's separators come from the forward: chunk
      // elimination and separator systems of the adjoint alone (output
      // gradient over the cover counts, one right-hand side per channel),
      // then the re-solve of both with the adjoint's separators after its
      // summaries in the interface buffer.
      const PassPlan pa = seps_plan(L, W, cb, p);   // the adjoint's own plan
      if (interface_bytes(pa) > lay.iface_img) return SGWLS_E_WORKSPACE;
      PassGeom ga = pass_geom(direction, M, N, pa, p.stride);
      if (bt) {
        Batch b = *bt;
        b.x = bt->x2;
        b.iface = (long long)lay.iface_img;
        set_batch(ga, b);
      }
      hipError_t e = launch_pass(p.r, cb, p.prec, ybar, g, nullptr, c0, ga, pa, wp, lam_dev,
                                 p.lambda, iface, stream, kStageReduce | kStageInterface, nullptr);
      if (e != hipSuccess) return SGWLS_E_HIP;
      pl.us_out = iface + pa.sum_elems * pa.acc_bytes;
      bw.useps = useps;
      bw.zseps = zseps;
      useps += align_up(pa.u_elems * pa.acc_bytes);
      stages = kStageExpand;
    }
    hipError_t e = launch_pass(p.r, cb, p.prec, x, g, xbar, c0, geo, pl, wp, lam_dev, p.lambda,
                               iface, stream, stages, &bw);
    if (e != hipSuccess) return SGWLS_E_HIP;
    if (!dfr) {
      e = launch_bwd_fixup(bw.side, gbar, geo, bw.lpart, expand_blocks(geo, pl), grad_lambda,
                           first ? 0 : 1, stream);
      if (e != hipSuccess) return SGWLS_E_HIP;
    }
    first = false;
    gf = false;
    c0 += cb;
  }
  return SGWLS_OK;
}

// ---------------------------------------------------------------------------
// Batches.  The tuning table stores the batched variant under the key
// (0, 0, fp64, kind, 2, bucket of the total pixel count).
constexpr int kBatchDir = 2;

TuneKey batch_tune_key(int fp64, int kind, double pixels) {
  return TuneKey(0, 0, fp64, kind, kBatchDir, (int)std::lround(2.0 * std::log2(std::max(pixels, 1.0))));
}

// Images are grouped by precision (float32 groups first), channel block
// (images whose channel count is a multiple of 3 are filtered three channels
// at a time, sharing the guidance weights; the others one channel at a time)
// and radius: group k = (prec * 2 + (cb == 3)) * kBatchMaxR + (r - 1), one
// launch per group, stage and pass.
constexpr int kBatchGroups = 4 * kBatchMaxR;

struct BatchPlan {
  int B = 0, passes = 0, kind = 0, variant = 0;
  int fp64 = 0;                    // every image in float64 (the variant count and tuning key)
  std::vector<BatchDesc> tab;      // by group, then largest image first
  int first[kBatchGroups + 1] = {};  // images of group k: tab[first[k], first[k+1])
  std::vector<int> pre;            // [group][dir][stage][B + 1] unit prefix sums over
                                   // the images of that group, then the [B + 1]
                                   // tile prefix sums of the guidance transposes
  int totals[kBatchGroups][2][3] = {};
  int tiles_t = 0;                 // 32 x 32 tiles of all guidance transposes
  size_t pre_at(int k, int dir, int st) const { return (size_t)((k * 2 + dir) * 3 + st) * (B + 1); }
  size_t pre_tiles() const { return (size_t)kBatchGroups * 6 * (B + 1); }
  size_t off_tab = 0, off_pre = 0, off_tmp = 0, off_gt = 0, off_iface = 0, off_iface64 = 0,
         total = 0;
  static int group_prec(int k) { return k / (2 * kBatchMaxR); }
  static int group_cb(int k) { return (k / kBatchMaxR) % 2 ? 3 : 1; }
  static int group_r(int k) { return k % kBatchMaxR + 1; }
  // float32 one-channel groups run the chosen variant, the other groups
  // their only one
  int group_variant(int k) const { return group_prec(k) || group_cb(k) == 3 ? 0 : variant; }
  size_t group_iface(int k) const { return group_prec(k) ? off_iface64 : off_iface; }
};

// Images the persistent batched kernels take: stride 1, r <= kBatchMaxR and
// sides whose chunk count the batched wave solver holds with every batched
// variant's chunk height.  The others of a batch (larger radii, strides > 1,
// longer sides) run through the single-image filter in the same call.
constexpr int batch_min_R(int r) {
  int m = 1 << 20;
  for (int fp = 0; fp < 2; ++fp)
    for (int v = 0; v < batch_variant_count(fp); ++v) {
      const BatchVariant bv = batch_variant(v, fp);
      const int R = r == 1 ? bv.R1 : bv.R2;
      m = R < m ? R : m;
    }
  return m;
}
// Channel block of an image in the persistent kernels: 3 where the channel
// count allows it and the three-channel chunk height keeps the sides within
// the wave solver, else 1 where the one-channel heights do, else 0 (the
// single-image path).
int batch_cb(const sgwls_image& im, const sgwls_params& p) {
  if (p.stride != 1 || p.r > kBatchMaxR) return 0;
  const int side = std::max(im.M, im.N);
  auto fits = [&](int R) { return (side + R - 1) / R - 1 <= kWave * kBatchMM; };
  const int fp64 = resolved(p, 0).prec == SGWLS_P_FP64_PIVOT ? 1 : 0;
  if (im.C % 3 == 0 && fits(variants_of(p.r, 3, fp64).v[0].R)) return 3;
  return fits(batch_min_R(p.r)) ? 1 : 0;
}
bool batch_eligible(const sgwls_image& im, const sgwls_params& p) { return batch_cb(im, p) > 0; }

// Validates the batch and lays out its workspace (ws may be NULL: sizes only).
sgwls_status batch_plan(const sgwls_image* imgs, const sgwls_params* p, int B, int variant,
                        void* ws, BatchPlan& plan) {
  if (!imgs || !p || B < 1 || B > (1 << 20)) return SGWLS_E_ARG;
  const sgwls_params& p0 = p[0];
  for (int b = 0; b < B; ++b) {
    const sgwls_image& im = imgs[b];
    const sgwls_status st = validate_partitioned(im.C, im.M, im.N, &p[b]);
    if (st != SGWLS_OK) return st;
    if (p[b].iters != p0.iters || p[b].kind != p0.kind || p[b].prec != p0.prec) return SGWLS_E_ARG;
    if (p[b].stride != 1 || p[b].r > kBatchMaxR) return SGWLS_E_UNSUPPORTED;
    if (ws && (!im.f || !im.g || !im.u || (const float*)im.u == im.g)) return SGWLS_E_ARG;
  }
  // Precision of every image: AUTO resolves image by image.
  std::vector<int> prec(B);
  int all64 = 1;
  for (int b = 0; b < B; ++b) {
    prec[b] = resolved(p[b], 0).prec == SGWLS_P_FP64_PIVOT ? 1 : 0;
    all64 &= prec[b];
  }
  if (variant < 0 || variant >= batch_variant_count(all64)) return SGWLS_E_ARG;
  plan.B = B;
  plan.passes = 2 * p0.iters;
  plan.fp64 = all64;
  plan.kind = (int)p0.kind;
  plan.variant = variant;
  std::vector<int> cbk(B);
  for (int b = 0; b < B; ++b) cbk[b] = batch_cb(imgs[b], p[b]);
  auto group_of = [&](int b) { return (prec[b] * 2 + (cbk[b] == 3 ? 1 : 0)) * kBatchMaxR + p[b].r - 1; };
  std::vector<int> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (group_of(a) != group_of(b)) return group_of(a) < group_of(b);
    return (long long)imgs[a].C * imgs[a].M * imgs[a].N > (long long)imgs[b].C * imgs[b].M * imgs[b].N;
  });
  for (int k = 0; k <= kBatchGroups; ++k) plan.first[k] = 0;
  for (int b = 0; b < B; ++b)
    for (int k = group_of(b) + 1; k <= kBatchGroups; ++k) ++plan.first[k];
  plan.off_tab = 0;
  plan.off_pre = align_up(sizeof(BatchDesc) * B);
  plan.off_tmp = plan.off_pre + align_up(sizeof(int) * (kBatchGroups * 6 + 1) * (B + 1));
  size_t tmp_bytes = 0, gt_bytes = 0;
  for (int b = 0; b < B; ++b) {
    tmp_bytes += image_bytes(imgs[b].C, imgs[b].M, imgs[b].N);
    gt_bytes += image_bytes(1, imgs[b].M, imgs[b].N);
  }
  plan.off_gt = plan.off_tmp + tmp_bytes;
  plan.off_iface = plan.off_gt + gt_bytes;
  char* base = reinterpret_cast<char*>(ws);
  plan.tab.assign(B, BatchDesc{});
  plan.pre.assign((kBatchGroups * 6 + 1) * (B + 1), 0);
  size_t tmp_off = plan.off_tmp, gt_off = plan.off_gt;
  size_t iface_elems[2] = {0, 0};   // float32 and float64 interface regions
  long long units[kBatchGroups][2][3] = {}, tiles = 0;
  for (int t = 0; t < B; ++t) {
    const int b = order[t];
    const sgwls_image& im = imgs[b];
    const sgwls_params& pb = p[b];
    const int k = group_of(b);
    const int cb = cbk[b];
    if (cb == 0) return SGWLS_E_UNSUPPORTED;
    const BatchVariant bv = batch_variant(prec[b] ? 0 : variant, prec[b]);
    const Variant v3 = variants_of(p[b].r, 3, prec[b]).v[0];
    BatchDesc& D = plan.tab[t];
    D.f = im.f;
    D.g = im.g;
    D.u = im.u;
    D.tmp = ws ? reinterpret_cast<float*>(base + tmp_off) : nullptr;
    tmp_off += image_bytes(im.C, im.M, im.N);
    D.gT = ws ? reinterpret_cast<float*>(base + gt_off) : nullptr;
    gt_off += image_bytes(1, im.M, im.N);
    tiles += (long long)((im.M + 31) / 32) * ((im.N + 31) / 32);
    plan.pre[plan.pre_tiles() + t + 1] = (int)std::min<long long>(tiles, 0x7fffffff);
    D.C = im.C;
    D.M = im.M;
    D.N = im.N;
    D.r = pb.r;
    D.lam = pb.lambda;
    D.wp = weight_params(pb);
    D.OW = kWave - 2 * pb.r;
    const int R = cb == 3 ? v3.R : pb.r == 1 ? bv.R1 : bv.R2;
    const int Q = cb == 3 ? v3.Q : bv.Q;
    const int T2 = pb.r * (pb.r + 1) / 2;
    const int F = 2 * T2 + 2 * pb.r * cb + pb.r * pb.r;
    const int nblk = im.C / cb;
    long long sum_max = 0, us_max = 0;
    for (int dir = 0; dir < 2; ++dir) {
      // Both passes are column passes storing transposed: the row pass runs
      // on the transposed image (N x M) that the column pass leaves.
      PassGeom& g = D.geo[dir];
      g.L = dir == 0 ? im.M : im.N;
      g.W = dir == 0 ? im.N : im.M;
      g.sa = g.W;
      g.sb = 1;
      g.out_t = 1;
      g.plane = (long long)im.M * im.N;
      g.nK = strip_count(g.W, pb.r, 1);
      g.stride = 1;
      g.R = R;
      g.P = (g.L + R - 1) / R;
      const int n = g.P - 1;
      D.m[dir] = std::max(1, (n + kWave - 1) / kWave);
      if (n > kWave * kBatchMM) return SGWLS_E_UNSUPPORTED;   // too long for the wave solver
      D.nbx_red[dir] = (g.nK + kWave - 1) / kWave;
      D.nbx_exp[dir] = (g.W + D.OW - 1) / D.OW;
      D.nby[dir] = (g.P + Q - 1) / Q;
      sum_max = std::max(sum_max, (long long)g.P * F * g.nK);
      us_max = std::max(us_max, (long long)std::max(n, 1) * pb.r * cb * g.nK);
      // Prefix sums of the group's sub-table: entry t - first + 1 (units of
      // every channel block of the image).
      const bool split = g.P > 1;
      long long* un = units[k][dir];
      un[0] += split ? (long long)nblk * D.nbx_red[dir] * D.nby[dir] : 0;
      un[1] += split ? (long long)nblk * g.nK : 0;
      un[2] += (long long)nblk * D.nbx_exp[dir] * D.nby[dir];
      const int tl = t - plan.first[k];
      for (int st = 0; st < 3; ++st)
        plan.pre[plan.pre_at(k, dir, st) + tl + 1] = (int)std::min<long long>(un[st], 0x7fffffff);
    }
    D.sum_ch = sum_max;
    D.us_ch = us_max;
    size_t& ie = iface_elems[prec[b]];
    D.sum_base = (long long)ie;
    ie += (size_t)nblk * sum_max;
    D.us_base = (long long)ie;
    ie += (size_t)nblk * us_max;
  }
  for (int k = 0; k < kBatchGroups; ++k)
    for (int dir = 0; dir < 2; ++dir)
      for (int st = 0; st < 3; ++st) {
        if (units[k][dir][st] > 0x7fffffffLL) return SGWLS_E_SHAPE;
        plan.totals[k][dir][st] = (int)units[k][dir][st];
      }
  if (tiles > 0x7fffffffLL) return SGWLS_E_SHAPE;
  plan.tiles_t = (int)tiles;
  plan.off_iface64 = plan.off_iface + align_up(iface_elems[0] * 4);
  plan.total = plan.off_iface64 + align_up(iface_elems[1] * 8);
  return SGWLS_OK;
}

// Writes host bytes into device memory with kernels whose arguments carry
// the data: the copy is ordered on the stream, capturable into a graph and
// independent of the lifetime of the host buffer.
hipError_t upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const unsigned int* w = reinterpret_cast<const unsigned int*>(src);
  const size_t nw = (bytes + 3) / 4;
  for (size_t o = 0; o < nw; o += WordChunk::kWords) {
    WordChunk c{};
    c.n = (unsigned int)std::min<size_t>(WordChunk::kWords, nw - o);
    std::memcpy(c.w, w + o, std::min<size_t>(bytes - o * 4, (size_t)c.n * 4));
    hipError_t e = launch_write_words(reinterpret_cast<unsigned int*>(dst) + o, c, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// All launches of one batched filter call.
sgwls_status batch_enqueue(const BatchPlan& plan, void* ws, hipStream_t s) {
  char* base = reinterpret_cast<char*>(ws);
  BatchDesc* tab = reinterpret_cast<BatchDesc*>(base + plan.off_tab);
  int* pre = reinterpret_cast<int*>(base + plan.off_pre);
  if (upload_bytes(tab, plan.tab.data(), sizeof(BatchDesc) * plan.B, s) != hipSuccess ||
      upload_bytes(pre, plan.pre.data(), sizeof(int) * plan.pre.size(), s) != hipSuccess)
    return SGWLS_E_HIP;
  if (launch_batch_transpose(tab, pre + plan.pre_tiles(), plan.B, plan.tiles_t, s) != hipSuccess)
    return SGWLS_E_HIP;
  for (int q = 0; q < plan.passes; ++q) {
    const int dir = q % 2;
    for (int k = 0; k < kBatchGroups; ++k) {
      const int b0 = plan.first[k], nb = plan.first[k + 1] - b0;
      if (nb == 0) continue;
      if (launch_batch_pass(plan.group_variant(k), BatchPlan::group_prec(k), plan.kind,
                            BatchPlan::group_r(k), BatchPlan::group_cb(k), tab + b0,
                            pre + plan.pre_at(k, dir, 0),
                            pre + plan.pre_at(k, dir, 1), pre + plan.pre_at(k, dir, 2),
                            plan.totals[k][dir], nb, q, dir, base + plan.group_iface(k),
                            s) != hipSuccess)
        return SGWLS_E_HIP;
    }
  }
  return SGWLS_OK;
}

// Instantiated graphs of batched calls, keyed by stream, workspace and the
// full plan (tables included), most recent first.
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec;
};
constexpr size_t kGraphCacheMax = 8;
std::list<GraphEntry>& graph_cache() {
  static std::list<GraphEntry> c;
  return c;
}
std::mutex& graph_mutex() {
  static std::mutex m;
  return m;
}

std::string graph_key(const BatchPlan& plan, void* ws, hipStream_t s) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
  put(&s, sizeof(s));
  put(&ws, sizeof(ws));
  put(&plan.variant, sizeof(int));
  put(&plan.fp64, sizeof(int));
  put(&plan.kind, sizeof(int));
  put(&plan.passes, sizeof(int));
  put(plan.tab.data(), sizeof(BatchDesc) * plan.tab.size());
  put(plan.pre.data(), sizeof(int) * plan.pre.size());
  return k;
}

// Runs the call as a graph on a non-default stream that is not capturing
// (captured once per distinct call, replayed afterwards); eagerly otherwise.
sgwls_status batch_run(const BatchPlan& plan, void* ws, hipStream_t s) {
  // Prepare the persistent grid sizes outside any capture (no launch).
  const int none[3] = {0, 0, 0};
  for (int k = 0; k < kBatchGroups; ++k)
    if (plan.first[k + 1] > plan.first[k] &&
        launch_batch_pass(plan.group_variant(k), BatchPlan::group_prec(k), plan.kind,
                          BatchPlan::group_r(k), BatchPlan::group_cb(k), nullptr, nullptr, nullptr,
                          nullptr, none, 0, 0, 0, nullptr, s) != hipSuccess)
      return SGWLS_E_HIP;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s == nullptr || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return batch_enqueue(plan, ws, s);
  const std::string key = graph_key(plan, ws, s);
  std::lock_guard<std::mutex> lk(graph_mutex());
  auto& cache = graph_cache();
  for (auto it = cache.begin(); it != cache.end(); ++it)
    if (it->key == key) {
      cache.splice(cache.begin(), cache, it);
      return hipGraphLaunch(cache.front().exec, s) == hipSuccess ? SGWLS_OK : SGWLS_E_HIP;
    }
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return SGWLS_E_HIP;
  const sgwls_status st = batch_enqueue(plan, ws, s);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  if (st != SGWLS_OK || ec != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return st != SGWLS_OK ? st : SGWLS_E_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess || !exec) return SGWLS_E_HIP;
  cache.push_front(GraphEntry{key, exec});
  while (cache.size() > kGraphCacheMax) {
    (void)hipGraphExecDestroy(cache.back().exec);
    cache.pop_back();
  }
  return hipGraphLaunch(exec, s) == hipSuccess ? SGWLS_OK : SGWLS_E_HIP;
}

// Persisted tuning table: with SGWLS_TUNE_CACHE naming a file, the table is
// loaded from it at the first lookup of a process (when the file matches this
// library version and the current device's architecture; otherwise it is
// ignored) and saved to it after every autotune call.
std::string device_arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  const std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

const char* tune_cache_path() {
  const char* path = std::getenv("SGWLS_TUNE_CACHE");
  return path && *path ? path : nullptr;
}

void tune_cache_load_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* path = tune_cache_path();
    if (!path) return;
    const std::string arch = device_arch_name();
    if (!arch.empty()) (void)sgwls_tune_load(path, arch.c_str());
  });
}

void tune_cache_save() {
  const char* path = tune_cache_path();
  if (!path) return;
  const std::string arch = device_arch_name();
  if (!arch.empty()) (void)sgwls_tune_save(path, arch.c_str());
}

struct BatchSplit {
  std::vector<sgwls_image> im;    // persistent-kernel images
  std::vector<sgwls_params> pp;
  std::vector<int> rest;          // indices of the single-image-path images
};

sgwls_status batch_split(const sgwls_image* imgs, const sgwls_params* p, int B, BatchSplit& s) {
  if (!imgs || !p || B < 1 || B > (1 << 20)) return SGWLS_E_ARG;
  for (int b = 0; b < B; ++b) {
    const sgwls_status st = sgwls_validate(imgs[b].C, imgs[b].M, imgs[b].N, &p[b]);
    if (st != SGWLS_OK) return st;
    if (p[b].iters != p[0].iters || p[b].kind != p[0].kind || p[b].prec != p[0].prec)
      return SGWLS_E_ARG;
    if (p[b].prec == SGWLS_P_FP32_DELTA) return SGWLS_E_UNSUPPORTED;
    if (batch_eligible(imgs[b], p[b])) {
      s.im.push_back(imgs[b]);
      s.pp.push_back(p[b]);
    } else {
      s.rest.push_back(b);
    }
  }
  return SGWLS_OK;
}

// Workspace of the single-image-path images (run one after another).
size_t batch_rest_bytes(const sgwls_image* imgs, const sgwls_params* p, const BatchSplit& s) {
  size_t need = 0;
  for (int b : s.rest)
    need = std::max(need, sgwls_workspace_bytes(imgs[b].C, imgs[b].M, imgs[b].N, &p[b], 0));
  return need;
}

double batch_pixels(const sgwls_image* imgs, int B) {
  double px = 0.0;
  for (int b = 0; b < B; ++b) px += (double)imgs[b].C * imgs[b].M * imgs[b].N;
  return px;
}

}  // namespace

sgwls::NoFusedScope::NoFusedScope() { ++t_no_fused; }
sgwls::NoFusedScope::~NoFusedScope() { --t_no_fused; }

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
  if (p->prec != SGWLS_P_FP32 && p->prec != SGWLS_P_FP64_PIVOT && p->prec != SGWLS_P_FP32_DELTA &&
      p->prec != SGWLS_P_AUTO)
    return SGWLS_E_ARG;
  if (C < 1 || M < 2 * p->r + 1 || N < 2 * p->r + 1) return SGWLS_E_SHAPE;
  // kernels address pixels with 32-bit element offsets
  if (M > kMaxSide || N > kMaxSide || (long long)C * M * N > 0x7fffffffLL) return SGWLS_E_SHAPE;
  if (p->r > kMaxR) return SGWLS_E_UNSUPPORTED;
  if (p->prec == SGWLS_P_FP32_DELTA && p->r != 1) return SGWLS_E_UNSUPPORTED;
  return SGWLS_OK;
}

namespace {
// Validation for the entry points of the partitioned kernels, which take the
// precision as their float64 switch: the serial-strip mode is filter only.
sgwls_status validate_partitioned(int C, int M, int N, const sgwls_params* p) {
  const sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  return p->prec == SGWLS_P_FP32_DELTA ? SGWLS_E_UNSUPPORTED : SGWLS_OK;
}

// Geometry of a pass of the serial-strip mode: a column pass over an L x W
// image (the image for even passes, its transpose for odd ones) that stores
// its output transposed, so every pass reads along rows.
PassGeom delta_geom(int L, int W, int stride) {
  PassGeom geo{};
  geo.L = L;
  geo.W = W;
  geo.sa = W;
  geo.sb = 1;
  geo.plane = (long long)L * W;
  geo.nK = strip_count(W, 1, stride);
  geo.stride = stride;
  geo.R = L;
  geo.P = 1;
  geo.out_t = 1;
  return geo;
}
}  // namespace

sgwls_precision sgwls_resolve_precision(const sgwls_params* p, int want_lambda_grad) {
  if (!p) return (sgwls_precision)-1;
  return resolved(*p, want_lambda_grad).prec;
}

size_t sgwls_workspace_bytes(int C, int M, int N, const sgwls_params* p, int save_for_backward) {
  return sgwls_workspace_bytes_nchw(1, C, M, N, p, save_for_backward);
}

size_t sgwls_workspace_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p,
                                  int save_for_backward) {
  if (B < 1 || sgwls_validate(C, M, N, p) != SGWLS_OK) return 0;
  const sgwls_params pr = resolved(*p, save_for_backward ? 1 : 0);
  p = &pr;
  if (p->prec == SGWLS_P_FP32_DELTA)   // one image; + slack to align the strip buffer
    return B == 1 ? sync_bytes(1, M, N) + image_bytes(C, M, N) + image_bytes(1, M, N) +
                        delta_buffer_bytes(C, M, N, p->stride) + kAlign
                  : 0;
  return sync_bytes(B, M, N) +
         (size_t)B * (image_bytes(C, M, N) + image_bytes(1, M, N) + iface_bytes_all(C, M, N, *p));
}

sgwls_status sgwls_pass_stages(int stages, int direction, const float* x, const float* g,
                               float* y, int C, int M, int N, const sgwls_params* p,
                               const float* lambda_dev, void* ws, size_t ws_bytes,
                               void* stream) {
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  const sgwls_params pr = resolved(*p, 0);
  p = &pr;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if ((stages & kStageAll) == 0 || stages > (kStageAll | kStageTransposeOut)) return SGWLS_E_ARG;
  if ((stages & kStageTransposeOut) &&
      (direction != 0 || p->stride != 1 || !frames_supported(C, p->r, p->stride, p->prec)))
    return SGWLS_E_UNSUPPORTED;
  if (!x || !g || !y || y == x || (const float*)y == g) return SGWLS_E_ARG;
  const size_t need = pass_iface_bytes(direction, C, M, N, *p);
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  clear_hip_error();
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
  return sgwls_filter_nchw(f, g, u, 1, C, M, N, p, lambda_dev, saved, ws, ws_bytes, stream);
}

sgwls_status sgwls_filter_status(void* ws, void* stream) {
  if (!ws) return SGWLS_E_ARG;
  clear_hip_error();
  unsigned int v = 0;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess ||
      hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
    return SGWLS_E_HIP;
  if (v != kSyncErrMagic) return SGWLS_OK;
  const unsigned int zero = 0;
  (void)hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice);
  return SGWLS_E_HIP;
}

// sgwls_filter_nchw, with the separator solutions of every pass written to
// seps (B images, per-image layout of seps_image_bytes) when it is non-NULL.
static sgwls_status filter_nchw_core(const float* f, const float* g, float* u, int B, int C,
                                     int M, int N, const sgwls_params* p,
                                     const float* lambda_dev, float* saved, char* seps,
                                     void* ws, size_t ws_bytes, void* stream) {
  sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (B < 1) return SGWLS_E_SHAPE;
  // Saved pass inputs feed a backward that may ask for the lambda gradient.
  const sgwls_params pr = resolved(*p, saved ? 1 : 0);
  p = &pr;
  if (!f || !g || !u || (const float*)u == g) return SGWLS_E_ARG;
  if (p->prec == SGWLS_P_FP32_DELTA) {
    // Serial-strip solves: no saved pass inputs (there is no backward in
    // this mode), one image.  As for the partitioned kernels, every pass is a
    // column pass storing transposed: pass 2t reads the image (guidance g)
    // and writes tmp (N x M), pass 2t+1 reads tmp (guidance g^T) and writes u.
    if (saved || B != 1) return SGWLS_E_UNSUPPORTED;
    const size_t img = image_bytes(C, M, N), gimg = image_bytes(1, M, N);
    const size_t sb = sync_bytes(1, M, N);
    if (!ws || ws_bytes < sb + img + gimg + delta_buffer_bytes(C, M, N, p->stride) + kAlign)
      return SGWLS_E_WORKSPACE;
    clear_hip_error();
    hipStream_t s = (hipStream_t)stream;
    char* base = reinterpret_cast<char*>(ws) + sb;
    float* tmp = reinterpret_cast<float*>(base);
    float* gT = reinterpret_cast<float*>(base + img);
    // the strip buffer holds 16-byte records: start it on an aligned address
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(base) + img + gimg;
    float* buf = reinterpret_cast<float*>((b0 + kAlign - 1) / kAlign * kAlign);
    if (launch_transpose(g, gT, M, N, s) != hipSuccess) return SGWLS_E_HIP;
    const WeightParams wp = weight_params(*p);
    const int passes = 2 * p->iters;
    const float* x = f;
    for (int q = 0; q < passes; ++q) {
      const bool even = q % 2 == 0;
      float* y = even ? tmp : u;
      if (launch_delta_pass(x, even ? g : gT, y, C,
                            even ? delta_geom(M, N, p->stride) : delta_geom(N, M, p->stride), wp,
                            lambda_dev, p->lambda, buf, s) != hipSuccess)
        return SGWLS_E_HIP;
      x = y;
    }
    return SGWLS_OK;
  }
  // Workspace: the synchronisation area, B intermediate images, B transposed
  // guidance planes, then B per-image interface buffers.
  const size_t img = image_bytes(C, M, N), gimg = image_bytes(1, M, N);
  const size_t iface_img = iface_bytes_all(C, M, N, *p);
  const size_t nb = (size_t)B;
  const size_t sb = sync_bytes(B, M, N);
  if (!ws || ws_bytes < sb + nb * (img + gimg + iface_img)) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  hipStream_t s = (hipStream_t)stream;
  unsigned int* sync = reinterpret_cast<unsigned int*>(ws);
  char* base = reinterpret_cast<char*>(ws) + sb;
  float* tmp = reinterpret_cast<float*>(base);
  float* gT = reinterpret_cast<float*>(base + nb * img);
  void* iface = base + nb * (img + gimg);
  const size_t plane = (size_t)C * M * N;
  const int passes = 2 * p->iters;
  // Per-image strides (floats): inputs and outputs C*M*N apart, the
  // intermediate images img/4 apart, the saved pass inputs 2T*C*M*N apart
  // (image b, pass q at (b*2T + q)*C*M*N), guidance planes (and their
  // transposes, written plane after plane) M*N apart.
  const long long sx = (long long)plane, ss = (long long)passes * (long long)plane;
  const long long stmp = (long long)(img / sizeof(float));
  auto stride_of = [&](const float* a) -> long long {
    if (saved && a >= saved && a < saved + (size_t)ss) return ss;
    return a == tmp ? stmp : sx;
  };
  auto batch = [&](const float* x, const float* y) {
    Batch b;
    b.n = B;
    b.x = stride_of(x);
    b.y = stride_of(y);
    b.g = (long long)M * N;
    b.iface = (long long)iface_img;
    return b;
  };
  // Pass 0's input is f itself; with saved separators the backward takes f,
  // so saved[0] is not written.
  if (saved && !seps && hipMemcpy2DAsync(saved, sizeof(float) * ss, f, sizeof(float) * plane,
                                sizeof(float) * plane, nb, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return SGWLS_E_HIP;
  // Strided forward calls without saved inputs also run as frames: their
  // column passes read directly and store through the LDS accumulators.
  if (frames_supported(C, p->r, p->stride, p->prec) || (p->stride != 1 && !saved)) {
    // Every pass is a column pass that stores its output transposed: pass 2t
    // reads the image (M x N), pass 2t+1 its transpose (N x M) -- the row pass
    // -- and writes the image layout again.  Without saved, pass 2t writes tmp
    // and pass 2t+1 writes u; with saved, pass q writes saved[q+1] (so odd
    // entries hold transposed images) and the last pass writes u.
    // One-launch passes: the transpose of g also clears the error word and
    // both counter banks.
    OneCtl one{};
    OneCtl* onep = nullptr;
    int nzero = 0;
    const int fuse = seps ? 0 : one_launch_mode();
    const long long zseps = seps ? (long long)seps_image_bytes(C, M, N, *p) : 0;
    char* sepr = nullptr;   // the separator regions, after the transposed guidance
    if (seps) {
      gT = reinterpret_cast<float*>(seps);
      sepr = seps + seps_guidance_bytes(B, M, N);
    }
    if (fuse && p->stride == 1) {
      one.full = fuse == 1;
      one.err = sync;
      one.banks = sync + kSyncHead / sizeof(unsigned int);
      one.counters = sync_counters(B, M, N);
      one.bank = 0;
      one.zeroed[0] = one.zeroed[1] = true;
      one.limit = one_launch_spin_limit();
      nzero = (int)(kSyncHead / sizeof(unsigned int)) + 2 * one.bank_words();
      onep = &one;
    }
    // The guidance transposed for the row passes: by pass 0's re-solve, from
    // the tile it stages for its transposed store (stride 1, three launches
    // per pass, and no separators stored by that re-solve); else by a
    // transpose of its own, which also clears the fused passes' words.
    const bool gt_pass0 =
        !onep && p->stride == 1 &&
        (!seps || forward_cut_like_backward(p->r, channel_block(C), p->prec));
    if (!gt_pass0 &&
        launch_transpose(g, gT, M, N, s, B, 0, onep ? sync : nullptr, nzero) != hipSuccess)
      return SGWLS_E_HIP;
    const float* x = saved && !seps ? saved : f;
    size_t soff = 0;
    for (int q = 0; q < passes; ++q) {
      const bool even = q % 2 == 0;
      float* y = q == passes - 1 ? u : saved ? saved + (size_t)(q + 1) * plane : even ? tmp : u;
      const Batch bt = batch(x, y);
      st = enqueue_pass(0, x, even ? g : gT, y, C, even ? M : N, even ? N : M, *p, lambda_dev,
                        iface, s, kStageAll | kStageTransposeOut, -1, &bt, onep,
                        seps ? sepr + soff : nullptr, zseps, gt_pass0 && q == 0 ? gT : nullptr);
      if (st != SGWLS_OK) return st;
      if (seps) soff += seps_pass_bytes(q, C, M, N, *p);
      x = y;
    }
    return SGWLS_OK;
  }
  if (seps) return SGWLS_E_UNSUPPORTED;
  // Pass q reads x_q and writes x_{q+1}; x_0 = f and x_{2T} = u.  With saved,
  // x_q lives in saved[q] (q < 2T); otherwise passes ping-pong between tmp
  // and u so that the last one lands in u.
  const float* x = saved ? saved : f;
  for (int q = 0; q < passes; ++q) {
    float* y;
    if (q == passes - 1) y = u;
    else if (saved) y = saved + (size_t)(q + 1) * plane;
    else y = ((passes - q) % 2 == 0) ? tmp : u;
    const Batch bt = batch(x, y);
    st = enqueue_pass(q % 2, x, g, y, C, M, N, *p, lambda_dev, iface, s, kStageAll, -1, &bt);
    if (st != SGWLS_OK) return st;
    x = y;
  }
  return SGWLS_OK;
}

sgwls_status sgwls_filter_nchw(const float* f, const float* g, float* u, int B, int C, int M,
                               int N, const sgwls_params* p, const float* lambda_dev,
                               float* saved, void* ws, size_t ws_bytes, void* stream) {
  return filter_nchw_core(f, g, u, B, C, M, N, p, lambda_dev, saved, nullptr, ws, ws_bytes,
                          stream);
}

size_t sgwls_separator_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p) {
  if (B < 1 || validate_partitioned(C, M, N, p) != SGWLS_OK) return 0;
  return seps_total_bytes(B, C, M, N, resolved(*p, 1));
}

sgwls_status sgwls_filter_nchw_seps(const float* f, const float* g, float* u, int B, int C,
                                    int M, int N, const sgwls_params* p,
                                    const float* lambda_dev, float* saved, void* seps,
                                    size_t seps_bytes, void* ws, size_t ws_bytes, void* stream) {
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (B < 1) return SGWLS_E_SHAPE;
  if (!saved || !seps || (const float*)u == f) return SGWLS_E_ARG;   // f is kept as pass 0's input
  const size_t need = seps_total_bytes(B, C, M, N, resolved(*p, 1));
  if (need == 0) return SGWLS_E_UNSUPPORTED;
  if (seps_bytes < need) return SGWLS_E_WORKSPACE;
  return filter_nchw_core(f, g, u, B, C, M, N, p, lambda_dev, saved,
                          reinterpret_cast<char*>(seps), ws, ws_bytes, stream);
}

int sgwls_variant_count(int r, int channel_block, int prec) {
  if (r < 1 || r > kMaxR || (channel_block != 1 && channel_block != 3) || (prec != 0 && prec != 1))
    return 0;
  return variants_of(r, channel_block, prec).n;
}

sgwls_status sgwls_tune_pin(int direction, int channel_block, int M, int N,
                            const sgwls_params* p, int variant) {
  sgwls_status st = validate_partitioned(channel_block, M, N, p);
  if (st != SGWLS_OK) return st;
  const sgwls_params pr = resolved(*p, 0);
  p = &pr;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if (channel_block != 1 && channel_block != 3) return SGWLS_E_ARG;
  const int nv = p->stride == 1 ? variants_of(p->r, channel_block, p->prec).n
                                 : strided_variant_count(p->r, channel_block, p->prec);
  if (variant < 0 || variant >= nv) return SGWLS_E_ARG;
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  const int kd = direction + (p->stride != 1 ? kStridedDir : 0);
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_table()[tune_key(p->r, channel_block, p->prec, (int)p->kind, kd, L, W)] = variant;
  return SGWLS_OK;
}

int sgwls_tune_query(int direction, int channel_block, int M, int N, const sgwls_params* p) {
  if (!p || (direction != 0 && direction != 1)) return -1;
  const sgwls_params pr = resolved(*p, 0);
  p = &pr;
  const int L = direction == 0 ? M : N, W = direction == 0 ? N : M;
  return tuned_variant(p->r, channel_block, p->prec, (int)p->kind,
                       direction + (p->stride != 1 ? kStridedDir : 0), L, W);
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
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  const sgwls_params pr = resolved(*p, 0);
  p = &pr;
  if (!x || !g || !y || y == x || (const float*)y == g || reps < 1) return SGWLS_E_ARG;
  const size_t need = std::max(pass_iface_bytes(0, C, M, N, *p), pass_iface_bytes(1, C, M, N, *p));
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  void* iface = ws;
  if (chosen)
    for (int i = 0; i < 4; ++i) chosen[i] = -1;
  tune_cache_load_once();
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
      const VariantSet vs = variants_of(p->r, cb, p->prec);
      const bool strided = p->stride != 1;
      const int nv = strided ? strided_variant_count(p->r, cb, p->prec) : vs.n;
      // With transposed frames the filter runs every pass as a direct column
      // pass storing transposed, over the M x N and the N x M frame, both
      // under the column-direction key: time exactly that.  Strided calls
      // without saved inputs run as frames too.
      const bool frames = dir == 0 && (strided || frames_supported(C, p->r, p->stride, p->prec));
      if (strided && (dir != 0 || nv < 2)) {
        if (chosen) chosen[dir * 2 + cbi] = 0;
        continue;
      }
      int best = 0;
      float best_ms = 0.0f;
      for (int v = 0; v < nv && result == SGWLS_OK; ++v) {
        if (!strided && frames && !vs.v[v].D) continue;
        auto run = [&]() {
          for (int f = 0; f < (frames ? 2 : 1); ++f) {
            const int Mf = f == 0 ? M : N, Nf = f == 0 ? N : M;
            const int Lf = dir == 0 ? Mf : Nf, Wf = dir == 0 ? Nf : Mf;
            const PassPlan pl = make_plan(Lf, Wf, p->r, cb, p->stride, p->prec, v);
            PassGeom geo = pass_geom(dir, Mf, Nf, pl, p->stride);
            geo.out_t = frames ? 1 : 0;
            const hipError_t e = launch_pass(p->r, cb, p->prec, x, g, y, c0, geo, pl, wp, nullptr,
                                             p->lambda, iface, s, kStageAll);
            if (e != hipSuccess) return e;
          }
          return hipSuccess;
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
        if (best_ms == 0.0f || ms < best_ms) { best = v; best_ms = ms; }
      }
      if (result != SGWLS_OK) break;
      {
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_table()[tune_key(p->r, cb, p->prec, (int)p->kind, dir + (strided ? kStridedDir : 0),
                              L, W)] = best;
      }
      if (chosen) chosen[dir * 2 + cbi] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result == SGWLS_OK) tune_cache_save();
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
    const bool batched = got == 7 && r == 0 && cb == 0 && dir == kBatchDir &&
                         (fp64 == 0 || fp64 == 1) && (kind == 0 || kind == 1) && v >= 0 &&
                         v < batch_variant_count(fp64);
    const bool single = got == 7 && r >= 1 && r <= kMaxR && (cb == 1 || cb == 3) &&
                        (fp64 == 0 || fp64 == 1) && (kind == 0 || kind == 1) &&
                        (dir == 0 || dir == 1) && v >= 0 && v < variants_of(r, cb, fp64).n;
    if (!batched && !single) {
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
  return sgwls_backward_workspace_bytes_nchw(1, C, M, N, p);
}

size_t sgwls_backward_workspace_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p) {
  if (B < 1 || validate_partitioned(C, M, N, p) != SGWLS_OK) return 0;
  // AUTO resolves per call (the lambda gradient decides): room for both.
  return std::max(bwd_layout(C, M, N, resolved(*p, 0), B).total,
                  bwd_layout(C, M, N, resolved(*p, 1), B).total);
}

sgwls_status sgwls_pass_backward(int direction, const float* x, const float* g,
                                 const float* ybar, float* xbar, float* gbar,
                                 double* grad_lambda, int C, int M, int N,
                                 const sgwls_params* p, const float* lambda_dev, void* ws,
                                 size_t ws_bytes, void* stream) {
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  const sgwls_params pr = resolved(*p, grad_lambda != nullptr);
  p = &pr;
  if (direction != 0 && direction != 1) return SGWLS_E_ARG;
  if (!x || !g || !ybar || !xbar || xbar == x || xbar == ybar || (const float*)xbar == g)
    return SGWLS_E_ARG;
  if (gbar && ((const float*)gbar == g || gbar == xbar || (const float*)gbar == x ||
               (const float*)gbar == ybar))
    return SGWLS_E_ARG;
  const BwdLayout lay = bwd_layout(C, M, N, *p);
  if (!ws || ws_bytes < lay.total) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  bool first = true;
  return enqueue_pass_backward(direction, x, g, ybar, xbar, gbar, grad_lambda, C, M, N, *p,
                               lambda_dev, ws, lay, (hipStream_t)stream, first);
}

sgwls_status sgwls_backward(const float* g, const float* saved, const float* grad_u,
                            float* grad_f, float* grad_g, double* grad_lambda, int C, int M,
                            int N, const sgwls_params* p, const float* lambda_dev, void* ws,
                            size_t ws_bytes, void* stream) {
  return sgwls_backward_nchw(g, saved, grad_u, grad_f, grad_g, grad_lambda, 1, C, M, N, p,
                             lambda_dev, ws, ws_bytes, stream);
}

// sgwls_backward_nchw; with seps (written by sgwls_filter_nchw_seps) the
// passes take the pass solutions' separators from it and run in the
// precision that call ran in.
// f0: pass 0's input (the forward's f) when saved[0] was not written.
static sgwls_status backward_nchw_core(const float* g, const float* f0, const float* saved,
                                       const char* seps, const float* grad_u, float* grad_f,
                                       float* grad_g,
                                       double* grad_lambda, int B, int C, int M, int N,
                                       const sgwls_params* p, const float* lambda_dev, void* ws,
                                       size_t ws_bytes, void* stream) {
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (B < 1) return SGWLS_E_SHAPE;
  const sgwls_params pr = resolved(*p, seps ? 1 : grad_lambda != nullptr);
  p = &pr;
  if (!g || !saved || !grad_u || !grad_f || (const float*)grad_f == g ||
      (const float*)grad_f == saved || (const float*)grad_f == f0)
    return SGWLS_E_ARG;
  if (f0 && grad_g && (const float*)grad_g == f0) return SGWLS_E_ARG;
  if (grad_g && ((const float*)grad_g == g || grad_g == grad_f || (const float*)grad_g == grad_u ||
                 (const float*)grad_g == saved))
    return SGWLS_E_ARG;
  const BwdLayout lay = bwd_layout(C, M, N, *p, B);
  if (!ws || ws_bytes < lay.total) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  hipStream_t s = (hipStream_t)stream;
  char* base = reinterpret_cast<char*>(ws);
  float* tmp = reinterpret_cast<float*>(base + lay.img_off);
  const size_t plane = (size_t)C * M * N;
  const int passes = 2 * p->iters;
  // Per-image strides (floats): gradients and intermediates C*M*N apart,
  // saved pass inputs 2T*C*M*N apart, guidance planes M*N apart.
  Batch bt;
  bt.n = B;
  bt.x = (long long)passes * (long long)plane;
  bt.x2 = bt.y = (long long)plane;
  bt.g = bt.gb = (long long)M * N;
  // Passes in reverse order.  Pass q reads the gradient of its output (grad_u
  // for the last pass) and writes that of its input: into grad_f for even q,
  // tmp for odd q, so pass 0 ends in grad_f and grad_u may alias grad_f.
  // grad_lambda receives the sum over the B images (lambda is shared).
  bool first = true;
  if (frames_supported(C, p->r, p->stride, p->prec)) {
    // The saved inputs of odd (row) passes are transposed (see sgwls_filter).
    // Pass q runs as a column pass in its frame (q odd: the transposed image
    // with the transposed guidance) and stores the input gradient transposed,
    // i.e. in the frame of pass q-1; pass 0 stores it as the image.  The
    // guidance gradient of odd passes accumulates transposed and is added to
    // grad_g at the end.
    // With saved separators the forward's transposed guidance is in seps.
    const float* gT = seps ? reinterpret_cast<const float*>(seps)
                           : reinterpret_cast<float*>(base + lay.gt_off);
    float* gTacc = reinterpret_cast<float*>(base + lay.gtacc_off);
    float* yT = reinterpret_cast<float*>(base + lay.yt_off);
    if ((!seps && launch_transpose(g, reinterpret_cast<float*>(base + lay.gt_off), M, N, s, B) !=
                      hipSuccess) ||
        launch_transpose(grad_u, yT, M, N, s, B * C) != hipSuccess)
      return SGWLS_E_HIP;
    const float* ybar = yT;
    bool gfirst[2] = {true, true};
    const long long zseps = seps ? (long long)seps_image_bytes(C, M, N, *p) : 0;
    const char* sepr = seps ? seps + seps_guidance_bytes(B, M, N) : nullptr;
    size_t soff = 0;
    for (int q = 0; seps && q < passes - 1; ++q) soff += seps_pass_bytes(q, C, M, N, *p);
    // The fix-ups wait for the end: side terms accumulate per frame parity
    // and channel block, lambda partials stay per pass (see below).
    int nblk = 0;
    for (int c0 = 0; c0 < C; c0 += channel_block(C - c0)) ++nblk;
    bool side_first[2] = {true, true};
    size_t lpart_end = 0;
    for (int q = passes - 1; q >= 0; --q) {
      const bool odd = q % 2 == 1;
      float* xbar = (q % 2 == 0) ? grad_f : tmp;
      BwdDefer dfr{odd ? nblk : 0, side_first[odd ? 1 : 0], lpart_end};
      Batch bq = bt;
      const float* xq = saved + (size_t)q * plane;
      if (f0 && q == 0) {   // pass 0's input is f (C*M*N floats per image)
        xq = f0;
        bq.x = (long long)plane;
      }
      st = enqueue_pass_backward(0, xq, odd ? gT : g, ybar, xbar,
                                 grad_g ? (odd ? gTacc : grad_g) : nullptr, grad_lambda, C,
                                 odd ? N : M, odd ? M : N, *p, lambda_dev, ws, lay, s, first,
                                 &gfirst[odd ? 1 : 0], q > 0 ? 1 : 0, &bq,
                                 seps ? sepr + soff : nullptr, zseps, &dfr);
      if (st != SGWLS_OK) return st;
      lpart_end = dfr.lpart_off;
      side_first[odd ? 1 : 0] = false;
      if (seps && q > 0) soff -= seps_pass_bytes(q - 1, C, M, N, *p);
      ybar = xbar;
    }
    // Deferred fix-ups: each parity's accumulated side terms into its
    // guidance gradient (odd: the transposed accumulator, before it is added
    // to grad_g), then every lambda partial of the call in one fixed-order
    // reduction.
    float* side0 = reinterpret_cast<float*>(base + lay.side_off);
    for (int par = 0; grad_g && par < 2; ++par) {
      const int L = par ? N : M, W = par ? M : N;   // the frame of the parity's passes
      for (int c0 = 0, blk = 0; c0 < C; ++blk) {
        const int cb = channel_block(C - c0);
        const PassPlan pl = make_plan(L, W, p->r, cb, 1, p->prec, 0, kModeBackward);
        PassGeom geo = pass_geom(0, L, W, pl, 1);
        Batch b = bt;
        b.side = (long long)lay.side_img;
        set_batch(geo, b);
        if (launch_bwd_fixup(side0 + (size_t)(par * nblk + blk) * lay.side_set,
                             par ? gTacc : grad_g, geo, nullptr, 0, nullptr, 0, s) != hipSuccess)
          return SGWLS_E_HIP;
        c0 += cb;
      }
    }
    if (grad_lambda) {
      PassGeom one_image{};
      one_image.P = 1;
      if (launch_bwd_fixup(nullptr, nullptr, one_image,
                           reinterpret_cast<const double*>(base + lay.lpart_off), (int)lpart_end,
                           grad_lambda, 0, s) != hipSuccess)
        return SGWLS_E_HIP;
    }
    if (grad_g && launch_transpose(gTacc, grad_g, N, M, s, B, 1) != hipSuccess) return SGWLS_E_HIP;
    return SGWLS_OK;
  }
  if (seps) return SGWLS_E_UNSUPPORTED;
  const float* ybar = grad_u;
  for (int q = passes - 1; q >= 0; --q) {
    float* xbar = (q % 2 == 0) ? grad_f : tmp;
    st = enqueue_pass_backward(q % 2, saved + (size_t)q * plane, g, ybar, xbar, grad_g,
                               grad_lambda, C, M, N, *p, lambda_dev, ws, lay, s, first, nullptr, 0,
                               &bt);
    if (st != SGWLS_OK) return st;
    ybar = xbar;
  }
  return SGWLS_OK;
}

// The persistent-kernel part of a batch (every image eligible).
sgwls_status sgwls_backward_nchw(const float* g, const float* saved, const float* grad_u,
                                 float* grad_f, float* grad_g, double* grad_lambda, int B, int C,
                                 int M, int N, const sgwls_params* p, const float* lambda_dev,
                                 void* ws, size_t ws_bytes, void* stream) {
  return backward_nchw_core(g, nullptr, saved, nullptr, grad_u, grad_f, grad_g, grad_lambda, B,
                            C, M, N, p, lambda_dev, ws, ws_bytes, stream);
}

sgwls_status sgwls_backward_nchw_seps(const float* g, const float* f, const float* saved,
                                      const void* seps, size_t seps_bytes,
                                      const float* grad_u, float* grad_f,
                                      float* grad_g, double* grad_lambda, int B, int C, int M,
                                      int N, const sgwls_params* p, const float* lambda_dev,
                                      void* ws, size_t ws_bytes, void* stream) {
  sgwls_status st = validate_partitioned(C, M, N, p);
  if (st != SGWLS_OK) return st;
  if (B < 1) return SGWLS_E_SHAPE;
  if (!seps || !f) return SGWLS_E_ARG;
  const size_t need = seps_total_bytes(B, C, M, N, resolved(*p, 1));
  if (need == 0) return SGWLS_E_UNSUPPORTED;
  if (seps_bytes < need) return SGWLS_E_WORKSPACE;
  return backward_nchw_core(g, f, saved, reinterpret_cast<const char*>(seps), grad_u, grad_f,
                            grad_g, grad_lambda, B, C, M, N, p, lambda_dev, ws, ws_bytes,
                            stream);
}

static size_t batched_core_bytes(const sgwls_image* imgs, const sgwls_params* p, int B) {
  if (!imgs || !p || B < 1) return 0;
  BatchPlan probe;
  if (batch_plan(imgs, p, B, 0, nullptr, probe) != SGWLS_OK) return 0;
  size_t need = 0;
  for (int v = 0; v < batch_variant_count(probe.fp64); ++v) {
    BatchPlan plan;
    if (batch_plan(imgs, p, B, v, nullptr, plan) != SGWLS_OK) return 0;
    need = std::max(need, plan.total);
  }
  return need;
}

int sgwls_batched_variant_count(int prec) {
  if (prec != 0 && prec != 1) return 0;
  return batch_variant_count(prec);
}

size_t sgwls_batched_workspace_bytes(const sgwls_image* imgs, const sgwls_params* p, int B) {
  BatchSplit sp;
  if (batch_split(imgs, p, B, sp) != SGWLS_OK) return 0;
  size_t core = 0;
  if (!sp.im.empty()) {
    core = batched_core_bytes(sp.im.data(), sp.pp.data(), (int)sp.im.size());
    if (core == 0) return 0;
  }
  return align_up(core) + batch_rest_bytes(imgs, p, sp);
}

static sgwls_status batched_core_run(const sgwls_image* imgs, const sgwls_params* p, int B,
                                     int variant, void* ws, size_t ws_bytes, void* stream) {
  BatchPlan probe;
  sgwls_status st = batch_plan(imgs, p, B, 0, nullptr, probe);
  if (st != SGWLS_OK) return st;
  if (variant < 0) {
    tune_cache_load_once();
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto it = tune_table().find(batch_tune_key(probe.fp64, probe.kind, batch_pixels(imgs, B)));
    variant = it == tune_table().end() ? 0 : it->second;
  }
  if (variant >= batch_variant_count(probe.fp64)) return SGWLS_E_ARG;
  if (!ws || ws_bytes < batched_core_bytes(imgs, p, B)) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  BatchPlan plan;
  st = batch_plan(imgs, p, B, variant, ws, plan);
  if (st != SGWLS_OK) return st;
  return batch_run(plan, ws, (hipStream_t)stream);
}

sgwls_status sgwls_filter_batched_variant(const sgwls_image* imgs, const sgwls_params* p, int B,
                                          int variant, void* ws, size_t ws_bytes, void* stream) {
  BatchSplit sp;
  sgwls_status st = batch_split(imgs, p, B, sp);
  if (st != SGWLS_OK) return st;
  for (int b = 0; b < B; ++b)
    if (!imgs[b].f || !imgs[b].g || !imgs[b].u || (const float*)imgs[b].u == imgs[b].g)
      return SGWLS_E_ARG;
  const size_t need = sgwls_batched_workspace_bytes(imgs, p, B);
  if (need == 0) return SGWLS_E_ARG;
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  const size_t core = sp.im.empty() ? 0 : align_up(batched_core_bytes(sp.im.data(), sp.pp.data(),
                                                                      (int)sp.im.size()));
  if (!sp.im.empty()) {
    st = batched_core_run(sp.im.data(), sp.pp.data(), (int)sp.im.size(), variant, ws, core, stream);
    if (st != SGWLS_OK) return st;
  } else if (variant >= batch_variant_count(0)) {
    return SGWLS_E_ARG;
  }
  char* rest_ws = reinterpret_cast<char*>(ws) + core;
  for (int b : sp.rest) {
    st = sgwls_filter(imgs[b].f, imgs[b].g, imgs[b].u, imgs[b].C, imgs[b].M, imgs[b].N, &p[b],
                      nullptr, nullptr, rest_ws, ws_bytes - core, stream);
    if (st != SGWLS_OK) return st;
  }
  return SGWLS_OK;
}

size_t sgwls_interpolate_workspace_bytes(int C, int M, int N, const sgwls_params* p) {
  if (C < 1 || C >= (1 << 20)) return 0;
  const size_t inner = sgwls_workspace_bytes(C + 1, M, N, p, 0);
  return inner ? image_bytes(C + 1, M, N) + inner : 0;
}

sgwls_status sgwls_interpolate(const float* f, const float* h, const float* g, float* u, int C,
                               int M, int N, const sgwls_params* p, const float* lambda_dev,
                               void* ws, size_t ws_bytes, void* stream) {
  if (C < 1 || C >= (1 << 20)) return SGWLS_E_ARG;
  sgwls_status st = sgwls_validate(C + 1, M, N, p);
  if (st != SGWLS_OK) return st;
  if (!f || !h || !g || !u || (const float*)u == g || (const float*)u == h) return SGWLS_E_ARG;
  const size_t stack = image_bytes(C + 1, M, N);
  const size_t need = sgwls_interpolate_workspace_bytes(C, M, N, p);
  if (!ws || ws_bytes < need) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  hipStream_t s = (hipStream_t)stream;
  // [S(f); S(h)] by one filter call over the stacked planes, filtered in
  // place; the filter's workspace comes first (its synchronisation area at
  // the start of ws), the stacked planes after it.
  const size_t inner = need - stack;
  float* X = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + inner);
  const size_t plane = (size_t)M * N;
  if (hipMemcpyAsync(X, f, sizeof(float) * C * plane, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(X + C * plane, h, sizeof(float) * plane, hipMemcpyDeviceToDevice, s) !=
          hipSuccess)
    return SGWLS_E_HIP;
  st = sgwls_filter(X, g, X, C + 1, M, N, p, lambda_dev, nullptr, ws, inner, stream);
  if (st != SGWLS_OK) return st;
  return launch_divide_planes(X, X + C * plane, u, C, (long long)plane, s) == hipSuccess
             ? SGWLS_OK
             : SGWLS_E_HIP;
}

sgwls_status sgwls_filter_batched(const sgwls_image* imgs, const sgwls_params* p, int B,
                                  void* ws, size_t ws_bytes, void* stream) {
  return sgwls_filter_batched_variant(imgs, p, B, -1, ws, ws_bytes, stream);
}

static sgwls_status autotune_batched_core(const sgwls_image* imgs, const sgwls_params* p, int B,
                                          void* ws, size_t ws_bytes, void* stream, int reps,
                                          int* chosen);

sgwls_status sgwls_autotune_batched(const sgwls_image* imgs, const sgwls_params* p, int B,
                                    void* ws, size_t ws_bytes, void* stream, int reps,
                                    int* chosen) {
  BatchSplit sp;
  sgwls_status st = batch_split(imgs, p, B, sp);
  if (st != SGWLS_OK) return st;
  if (reps < 1) return SGWLS_E_ARG;
  if (!ws || ws_bytes < sgwls_batched_workspace_bytes(imgs, p, B)) return SGWLS_E_WORKSPACE;
  if (sp.im.empty()) {   // nothing for the persistent kernels to tune
    if (chosen) *chosen = 0;
    return SGWLS_OK;
  }
  return autotune_batched_core(sp.im.data(), sp.pp.data(), (int)sp.im.size(), ws, ws_bytes,
                               stream, reps, chosen);
}

static sgwls_status autotune_batched_core(const sgwls_image* imgs, const sgwls_params* p, int B,
                                          void* ws, size_t ws_bytes, void* stream, int reps,
                                          int* chosen) {
  BatchPlan probe;
  sgwls_status st = batch_plan(imgs, p, B, 0, nullptr, probe);
  if (st != SGWLS_OK) return st;
  if (reps < 1) return SGWLS_E_ARG;
  if (!ws || ws_bytes < batched_core_bytes(imgs, p, B)) return SGWLS_E_WORKSPACE;
  clear_hip_error();
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SGWLS_E_HIP;
  }
  int best = 0;
  float best_ms = 0.0f;
  sgwls_status result = SGWLS_OK;
  for (int v = 0; v < batch_variant_count(probe.fp64) && result == SGWLS_OK; ++v) {
    BatchPlan plan;
    result = batch_plan(imgs, p, B, v, ws, plan);
    if (result != SGWLS_OK) break;
    result = batch_enqueue(plan, ws, s);   // warm-up
    if (result != SGWLS_OK || hipEventRecord(e0, s) != hipSuccess) { result = SGWLS_E_HIP; break; }
    for (int i = 0; i < reps && result == SGWLS_OK; ++i) result = batch_enqueue(plan, ws, s);
    float ms = 0.0f;
    if (result != SGWLS_OK || hipEventRecord(e1, s) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      if (result == SGWLS_OK) result = SGWLS_E_HIP;
      break;
    }
    if (v == 0 || ms < best_ms) { best = v; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != SGWLS_OK) return result;
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_table()[batch_tune_key(probe.fp64, probe.kind, batch_pixels(imgs, B))] = best;
  }
  tune_cache_save();
  if (chosen) *chosen = best;
  return SGWLS_OK;
}

int sgwls_batched_graph_count(void) {
  std::lock_guard<std::mutex> lk(graph_mutex());
  return (int)graph_cache().size();
}

void sgwls_batched_graph_clear(void) {
  std::lock_guard<std::mutex> lk(graph_mutex());
  for (auto& e : graph_cache()) (void)hipGraphExecDestroy(e.exec);
  graph_cache().clear();
}

}  // extern "C"
