// Internal declarations shared by the kernel translation units and the C ABI.
// Nothing here is part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#define DEV_HOST_INLINE __host__ __device__ inline

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
  float inv_sr2;               // exp: 1 / sigma_r^2 (derivative of the range factor)
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
  int out_t;        // 1: the output is stored transposed, pixel (a, b) at b*L + a
                    // (stride-1 column passes with direct reads only)
  // An NCHW batch of equal-shape images in one launch (blockIdx.z = image):
  // per-image strides, in floats, of the input x, the second source (the
  // backward's output gradient), the output y, the guidance g, the guidance
  // gradient and the backward side buffer; in bytes of the interface
  // buffers; in entries of the lambda partials.  nimg = 1 and zero strides
  // for one image.
  int nimg;
  long long zx, zx2, zy, zg, zgb, zside, zi;
  int zlpart;
  long long zu;     // bytes between images of the separator solutions (zi unless
                    // they are written to a buffer of their own)
};

// Image z of a batched launch: p moved by z * stride elements (or bytes).
template <typename T>
DEV_HOST_INLINE T* zmove(T* p, long long stride, int z) {
  return p ? p + (long long)z * stride : p;
}
template <typename T>
DEV_HOST_INLINE T* zmove_bytes(T* p, long long bytes, int z) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long long)z * bytes) : p;
}

// Per-image strides of a batched call (see PassGeom); n = 1: one image.
struct Batch {
  int n = 1;
  long long x = 0, x2 = 0, y = 0, g = 0, gb = 0, side = 0, iface = 0;
  int lpart = 0;
};
DEV_HOST_INLINE void set_batch(PassGeom& geo, const Batch& b) {
  geo.nimg = b.n;
  geo.zx = b.x;
  geo.zx2 = b.x2;
  geo.zy = b.y;
  geo.zg = b.g;
  geo.zgb = b.gb;
  geo.zside = b.side;
  geo.zi = b.iface;
  geo.zu = b.iface;
  geo.zlpart = b.lpart;
}

// Kernel variants: rows per chunk R (even) and chunks per block Q.  Stride-1
// passes may use any variant of their case; strided passes always use
// variant 0's R with Q = 1 (their tiles are wider).
struct Variant {
  int R, Q;
  int D;    // 1: the column pass reads chunks straight from global memory (no LDS tile)
};
constexpr int kMaxVariants = 12;
struct VariantSet {
  int n;
  Variant v[kMaxVariants];
  int MM;   // separators per lane handled by the wave interface solver
};

// Kernels of a pass: the forward solve, or its adjoint (two right-hand sides
// per channel: the recomputed pass solution and the adjoint solve).
constexpr int kModeForward = 0, kModeBackward = 1;
// The adjoint half of a backward pass on its own: chunk elimination and
// separator systems of the output gradient divided by the cover counts (one
// right-hand side per channel), in the backward's chunk shape; the backward
// re-solve then takes the pass solution's separators from the forward.
constexpr int kModeAdjoint = 2;

// The expand kernel keeps (r + CB) values per chunk element in registers, so
// R shrinks as r, the channel block and the precision grow.
constexpr VariantSet variants_of(int r, int cb, int fp64) {
  if (fp64) {
    // r = 1, three channels: six-row chunks first (0.290 against 0.315 ms for
    // four rows on 1080p RGB; eight rows need all 256 VGPRs and are slower)
    if (r == 1) return cb == 1 ? VariantSet{2, {{8, 4, 1}, {4, 4}}, 8} : VariantSet{3, {{6, 4, 1}, {4, 4, 1}, {4, 2}}, 8};
    if (r == 2) return cb == 1 ? VariantSet{1, {{4, 4, 1}}, 4} : VariantSet{1, {{2, 4, 1}}, 4};
    return VariantSet{1, {{2, 2, 1}}, 0};
  }
  // Variant 0 first; the row-pass tile loader keeps a lane per tile row, so
  // Q*R + 2 close to (and not above) 64 uses the lanes best.  Every tile
  // stays within 64 KB of LDS.
  if (r == 1)
    return cb == 1
               ? VariantSet{9, {{16, 4, 1}, {16, 3, 0}, {8, 7, 0}, {12, 5, 0}, {8, 4, 1},
                                {16, 4, 0}, {16, 2, 1}, {12, 4, 1}, {8, 4, 0}}, 8}
               : VariantSet{10, {{8, 4, 1}, {8, 7, 0}, {6, 9, 0}, {10, 5, 0}, {8, 2, 1},
                                 {6, 4, 1}, {10, 4, 1}, {8, 4, 0}, {8, 8, 1}, {4, 8, 1}}, 8};
  if (r == 2)
    return cb == 1 ? VariantSet{5, {{6, 4, 1}, {6, 9}, {4, 8, 1}, {4, 4}, {6, 4}}, 8}
                   : VariantSet{5, {{4, 4, 1}, {4, 8}, {4, 8, 1}, {4, 2}, {4, 4}}, 8};
  if (r == 3) return cb == 1 ? VariantSet{1, {{4, 2, 1}}, 0} : VariantSet{1, {{2, 2, 1}}, 0};
  return VariantSet{1, {{2, 2, 1}}, 0};
}

// Backward variants: 2*cb right-hand sides per element.
constexpr VariantSet bwd_variants_of(int r, int cb, int fp64) {
  if (fp64) {
    if (r == 1) return cb == 1 ? VariantSet{1, {{8, 4, 1}}, 8} : VariantSet{1, {{4, 4, 1}}, 8};
    if (r == 2) return VariantSet{1, {{2, 4, 1}}, 0};
    return VariantSet{1, {{2, 2, 1}}, 0};
  }
  if (r == 1)
    return cb == 1 ? VariantSet{3, {{8, 4, 1}, {8, 4}, {4, 4}}, 8}
                   : VariantSet{3, {{6, 4, 1}, {4, 4, 1}, {4, 4}}, 8};
  if (r == 2) return VariantSet{2, {{4, 4, 1}, {4, 4}}, 8};
  return VariantSet{1, {{2, 2, 1}}, 0};
}

// A forward variant reading its chunks directly and cut like variant 0 of the
// backward (whose interface then solves the backward's separators).
constexpr int forward_variant_cut_like_backward(int r, int cb, int fp64) {
  const VariantSet fw = variants_of(r, cb, fp64), bw = bwd_variants_of(r, cb, fp64);
  for (int v = 0; v < fw.n; ++v)
    if (fw.v[v].D && fw.v[v].R == bw.v[0].R) return v;
  return -1;
}
constexpr bool forward_cut_like_backward(int r, int cb, int fp64) {
  return forward_variant_cut_like_backward(r, cb, fp64) >= 0;
}

constexpr VariantSet variants_for(int mode, int r, int cb, int fp64) {
  return mode == kModeForward ? variants_of(r, cb, fp64) : bwd_variants_of(r, cb, fp64);
}

// Strided forward passes: variant 0 uses variant 0's R with one chunk (one
// wave) per block; variant 1 two chunks per block, so the transposed output
// of a block is 2R rows long instead of R; variant 2 (where R/2 is even)
// half-height chunks four to a block (more blocks, and 2R rows per block).
// A variant whose LDS accumulators exceed 64 KiB at the call's stride runs
// as variant 0.  Strided backward passes have variant 0 only.
struct StridedVariant {
  int R, Q;
};
constexpr int strided_half_R(int r, int cb, int fp64) {
  const int R0 = variants_of(r, cb, fp64).v[0].R;
  return (R0 >= 4 && (R0 / 2) % 2 == 0) ? R0 / 2 : 0;
}
constexpr int strided_variant_count(int r, int cb, int fp64, int mode = kModeForward) {
  return mode != kModeForward ? 1 : strided_half_R(r, cb, fp64) > 0 ? 3 : 2;
}
constexpr StridedVariant strided_variant(int r, int cb, int fp64, int v) {
  const int R0 = variants_of(r, cb, fp64).v[0].R;
  return v == 1 ? StridedVariant{R0, 2} : v == 2 ? StridedVariant{strided_half_R(r, cb, fp64), 4}
                                                 : StridedVariant{R0, 1};
}
constexpr size_t kStridedLdsMax = 65536;

// Synchronisation area at the start of the workspaces of sgwls_filter and
// sgwls_filter_nchw: the error word of the fused passes (kSyncErrMagic after
// a wait gave up; any other value means no error), then two banks of
// counters used by alternate fused passes (two counters per image and strip
// group; each launch zeroes the other bank for the next).
constexpr unsigned int kSyncErrMagic = 0x53475731u;
constexpr size_t kSyncHead = 256;
// Counters sit 256 bytes apart, so that the polls of different strip groups
// go to different memory channels.
constexpr int kCounterStride = 64;

// Host state of the one-launch passes of one call.
struct OneCtl {
  unsigned int* err;      // error word
  unsigned int* banks;    // two banks of bank_words() words
  long long counters;     // counters of each kind per bank (images x strip groups)
  int bank;               // bank of the next one-launch pass
  bool zeroed[2];         // whether each bank is known to be zero on the stream
  unsigned int limit;     // polls per wait before giving up
  bool full;              // expand in the same launch (else a launch of its own)
  DEV_HOST_INLINE int bank_words() const { return (int)(2 * counters * kCounterStride); }
  DEV_HOST_INLINE unsigned int* bank_ptr(int b) const { return banks + (size_t)b * bank_words(); }
};
// While a NoFusedScope lives, filter calls on this thread run three launches
// per pass whatever SGWLS_ONE_LAUNCH says (for callers whose workspace the
// user cannot read the fused passes' error word back from).
struct NoFusedScope {
  NoFusedScope();
  ~NoFusedScope();
  NoFusedScope(const NoFusedScope&) = delete;
  NoFusedScope& operator=(const NoFusedScope&) = delete;
};

// Synchronisation bytes of a call over B images of M x N (strip groups of 64
// strips across the wider frame).
inline size_t sync_bytes(int B, int M, int N) {
  const long long groups = (long long)B * ((M > N ? M : N) / 64 + 1);
  return kSyncHead + sizeof(unsigned int) * 4 * (size_t)kCounterStride * (size_t)groups;
}
inline long long sync_counters(int B, int M, int N) {
  return (long long)B * ((M > N ? M : N) / 64 + 1);
}

// Launch configuration of one (r, channel block, precision, stride, variant).
struct PassPlan {
  int mode;         // kModeForward or kModeBackward
  int nr;           // right-hand sides per element (cb, or 2*cb backward)
  int variant;      // index into variants_for(mode, r, cb, fp64)
  int R;            // rows per chunk
  int Q;            // chunks per reduce / expand block (one wave each)
  int P;            // chunks per subsystem
  int nK;           // strip centres
  int OW;           // output columns owned by one expand block
  int TB;           // LDS tile width (columns across the pass)
  int pitch;        // LDS row pitch (odd)
  int iface_m;      // separators per lane of the wave interface solver (0: serial solver)
  size_t sum_elems, u_elems;   // interface buffer sizes (elements)
  size_t g_elems;              // scratch of the long-run interface solver (elements)
  int long_nl;                 // lanes per strip of the long-run solver (64, 128 or 256)
  int mw_nl;                   // > 0: the register solver on mw_nl lanes per strip instead
  int acc_bytes;    // 4 (float) or 8 (double) interface element size
  OneCtl* one;      // set by the caller to allow the one-launch pass
  void* us_out;     // non-NULL: separator solutions here instead of after the summaries
};

// Cancellation-free float32 mode at r = 1 (sgwls_delta.hip): one serial
// solve per strip with pivots carried as their excess over the remaining
// coupling, channels in groups of kDeltaGroup.  The buffer holds one group's
// eliminated strips of the larger pass direction.
constexpr int kDeltaGroup = 4;
size_t delta_buffer_bytes(int C, int M, int N, int stride);
hipError_t launch_delta_pass(const float* x, const float* g, float* y, int C,
                             const PassGeom& geo, const WeightParams& wp, const float* lam_dev,
                             float lam_host, float* buf, hipStream_t s);

// Host-side planning (sgwls_plan.cpp).
int strip_count(int W, int r, int stride);
PassPlan make_plan(int L, int W, int r, int cb, int stride, int fp64, int variant,
                   int mode = kModeForward);
size_t interface_bytes(const PassPlan& pl);
// Largest interface_bytes over every variant of the case.
size_t interface_bytes_max(int L, int W, int r, int cb, int stride, int fp64,
                           int mode = kModeForward);
// Expand blocks of a plan (one double of the lambda gradient each).
int expand_blocks(const PassGeom& geo, const PassPlan& pl);

// Whether every channel block of a stride-1 request has direct-read variant 0
// forward and backward, so that passes can run as column passes of the image
// and of its transpose (the layout of saved pass inputs depends on this).
bool frames_supported(int C, int r, int stride, int fp64);

// Stages of one pass (bit mask): reduce, interface solve, expand.
constexpr int kStageReduce = 1, kStageInterface = 2, kStageExpand = 4, kStageAll = 7;
// With the stage mask: store the pass output transposed (see PassGeom::out_t).
constexpr int kStageTransposeOut = 8;


// Extra operands of a backward pass (all device pointers).
struct BwdArgs {
  const float* ybar;   // gradient of the pass output, C planes
  float* gbar;         // gradient of the guidance (NULL: not wanted)
  float* side;         // P x W floats: guidance-gradient terms of edges that cross chunk
                       // boundaries, for the pixels of the chunk above
  double* lpart;       // one partial lambda gradient per expand block (NULL: not wanted)
  int gacc;            // 1: add to gbar, 0: overwrite it
  int sacc;            // 1: add to side (terms of several passes), 0: overwrite it
  // Separators of the pass solution saved by the forward (layout of a forward
  // interface buffer's solutions, r x CB per separator), or NULL: then the
  // pass solves them itself (2 CB right-hand sides); with them the
  // interface buffer holds the adjoint's separators only (r x CB).
  const void* useps;
  long long zseps;     // bytes between the images of an NCHW batch in useps / seps_out
  // Forward passes: non-NULL to also store the pass solution at the chunk
  // separators of another cut of the subsystems (seps_R rows per chunk,
  // seps_n separators per strip), in the layout useps reads.
  void* seps_out;
  int seps_R, seps_n;
  // Forward column passes storing transposed: non-NULL to also store the
  // guidance transposed here (W x L, image z at z * zg floats).
  float* gT_out;
};

// Enqueue the stages in `stages` of one pass for channels [c0, c0+cb) of x
// into y.  `iface` must hold interface_bytes(plan).  For a backward plan, x is
// the saved pass input, y receives the input gradient and `bw` carries the
// rest.  Returns a hipError_t.
hipError_t launch_pass(int r, int cb, int fp64, const float* x, const float* g, float* y,
                       int c0, const PassGeom& geo, const PassPlan& plan,
                       const WeightParams& wp, const float* lam_dev, float lam_host,
                       void* iface, hipStream_t stream, int stages,
                       const BwdArgs* bw = nullptr);

// After the backward expand of a pass: add the side terms into gbar (when
// non-NULL) and reduce the nparts lambda partials into *glam (when both are
// non-NULL; lam_acc = 1 adds, 0 overwrites), in a fixed order.
hipError_t launch_bwd_fixup(const float* side, float* gbar, const PassGeom& geo,
                            const double* lpart, int nparts, double* glam, int lam_acc,
                            hipStream_t stream);

// ---------------------------------------------------------------------------
// Batches of uneven images (one channel per work unit, stride 1, r <= 2).
// Each stage of a pass is one persistent launch per radius over all images
// of that radius: its workgroups stride over the units (image, channel,
// block), so small and large images share the GPU.

constexpr int kBatchMaxR = 2;
constexpr int kBatchMM = 8;       // separators per lane of the batched wave solver
constexpr int kBatchVariants = 3;

// Rows per chunk for r = 1 and r = 2 and chunks per block (all variants of
// one precision share the block shape only within a variant).
struct BatchVariant {
  int R1, R2, Q;
};
constexpr BatchVariant batch_variant(int v, int fp64) {
  if (fp64) return BatchVariant{8, 4, 4};
  return v == 1 ? BatchVariant{8, 4, 4} : v == 2 ? BatchVariant{16, 6, 2} : BatchVariant{16, 6, 4};
}
constexpr int batch_variant_count(int fp64) { return fp64 ? 1 : kBatchVariants; }

// Device table entry of one image.
struct BatchDesc {
  const float* f;      // input, C x M x N
  const float* g;      // guidance, M x N
  float* u;            // output
  float* tmp;          // ping-pong image, transposed frame (workspace)
  float* gT;           // transposed guidance, N x M (workspace)
  int C, M, N, r;
  float lam;
  int pad0;
  WeightParams wp;
  PassGeom geo[2];     // column pass of the image (M x N) and of its transpose (N x M)
  int OW;              // output columns per expand block
  int m[2];            // separator blocks per lane of the interface solver
  int nbx_red[2], nbx_exp[2], nby[2];
  long long sum_base, us_base;   // interface buffers (elements of the accumulation type)
  long long sum_ch, us_ch;       // per-channel strides of those buffers
};

// Stages of one batched pass over the images of radius r filtered in blocks
// of cb channels (1, or 3 with the three-channel chunk shape; tab: their
// table entries, B of them); prefix = the (B+1) unit prefix sums of the
// stage's direction.
// With all totals 0 it launches nothing and only prepares the persistent
// grid sizes of the variant (a device query, not a stream operation).
hipError_t launch_batch_pass(int variant, int fp64, int kind, int r, int cb, const BatchDesc* tab,
                             const int* prefix_reduce, const int* prefix_iface,
                             const int* prefix_expand, const int totals[3], int B, int q,
                             int dir, void* iface, hipStream_t stream);
// dst (cols x rows) = transpose of src (rows x cols), `planes` planes; with
// accumulate, dst += the transpose.
hipError_t launch_transpose(const float* src, float* dst, int rows, int cols, hipStream_t stream,
                            int planes = 1, int accumulate = 0, unsigned int* zero = nullptr,
                            int nzero = 0);
// dst[0..n) = 0, ordered on the stream (no memset node in captured graphs).
hipError_t launch_zero_words(unsigned int* dst, int n, hipStream_t stream);

// u[c] = num[c] / den for c < C (planes of `plane` floats).
hipError_t launch_divide_planes(const float* num, const float* den, float* u, int C,
                                long long plane, hipStream_t stream);

// Transposed guidance of every image of a batch (pre_t: tile prefix sums).
hipError_t launch_batch_transpose(const BatchDesc* tab, const int* pre_t, int B, int tiles,
                                  hipStream_t stream);


// Up to kWords 32-bit words carried by value as kernel arguments.
struct WordChunk {
  static constexpr unsigned int kWords = 896;   // kernel arguments stay below 4 KiB
  unsigned int n;
  unsigned int w[kWords];
};
// dst[0..c.n) = c.w[0..c.n), ordered on the stream.
hipError_t launch_write_words(unsigned int* dst, const WordChunk& c, hipStream_t stream);

// Per-radius entry points (one translation unit each).
#define SGWLS_DECLARE_LAUNCH(RR)                                                            \
  hipError_t launch_pass_r##RR(int cb, int fp64, const float* x, const float* g, float* y, \
                               int c0, const PassGeom& geo, const PassPlan& plan,          \
                               const WeightParams& wp, const float* lam_dev,               \
                               float lam_host, void* iface, hipStream_t stream, int stages, \
                               const BwdArgs* bw);
SGWLS_DECLARE_LAUNCH(1)
SGWLS_DECLARE_LAUNCH(2)
SGWLS_DECLARE_LAUNCH(3)
SGWLS_DECLARE_LAUNCH(4)
#undef SGWLS_DECLARE_LAUNCH

}  // namespace sgwls
