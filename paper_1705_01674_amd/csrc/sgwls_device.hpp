// HIP kernels for one SG-WLS pass on gfx950 (MI355X), included by one
// translation unit per neighbourhood radius (sgwls_pass_r<r>.hip).
//
// One pass (Sec. 2.3 of Liu et al., ICCV 2017) solves, for every strip centre
// k, the subsystem A_s u = f of Eq. (5): A_s = I + lambda*L on the vector of
// s = (2r+1)L pixels built by the neighbourhood construction of Sec. 2.1, with
// the guidance weights of Eq. (2) on pairs at most r apart along the vector.
// The solutions are scattered back and averaged over the strips covering each
// pixel.
//
// A_s is symmetric positive definite with half-bandwidth r, so any exact
// elimination is admissible (Sec. 2.2 solves it with an r-band LU).  A single
// serial sweep per subsystem would leave the GPU idle (a 1080p column pass has
// 1918 subsystems of 3240 elements), so every subsystem is cut into chunks of
// R rows (R(2r+1) elements) and solved exactly by a partitioned (Schur
// complement) method in three kernels:
//
//   k_reduce     lanes = 64 adjacent strips, waves = Q consecutive chunks.  The
//                last r elements of every chunk but the last are a separator
//                block S_j.  Each lane eliminates its chunk interior I_j
//                (banded LDL^T with a right-looking (r+1)x(r+1) window) while
//                carrying the previous separator S_{j-1} as a border, and emits
//                the chunk's contribution to the Schur complement on the
//                separators.
//   k_interface  one wave per strip: the separator system is block tridiagonal
//                (r x r blocks, one per chunk boundary).  Each lane eliminates
//                a run of m consecutive separator blocks (the same bordered
//                elimination, one level up), the 64 remaining blocks are solved
//                by block parallel cyclic reduction across the lanes, and each
//                lane back-substitutes its run.  (A serial one-lane-per-strip
//                solver covers runs too long for registers.)
//   k_expand     same block shape as k_reduce: each lane re-solves its chunk
//                with both separators known, and the block averages the strips
//                covering each pixel in LDS in a fixed order (no atomics,
//                bitwise reproducible) before writing the pixels it owns.
//
// Image tiles are staged through LDS so that global loads and stores are
// contiguous in both pass directions; lanes then read their strip's pixels
// from LDS.  Weights and the band of A_s are recomputed from the guidance; no
// per-pixel intermediate goes to memory.
#pragma once

#include "sgwls_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace sgwls {
namespace {

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// Arithmetic helpers.

// Guidance value of tile rows outside the subsystem (see load_tile), and the
// guidance difference from which an edge is taken to reach such a row.
constexpr float kSentinel = 1.0e30f;
constexpr float kSentinelGap = 1.0e29f;

// Range factor of Eq. (2); the spatial factor is folded into lambda*S(d).
// exp: 2^(-dG^2 * log2(e)/(2 sigma_r^2)); frac: 1/(|dG|^alpha_r + eps) with
// |dG|^alpha_r = 2^(alpha_r log2|dG|).  Hardware exp2/log2/rcp (about 1 ulp).
// An edge to a row outside the image gets 0: exp underflows (dG^2 is
// infinite), and frac is set to 0 from |dG| >= kSentinelGap (with a small
// alpha_r its formula would otherwise couple the border pixels to the
// padding).
template <int KIND>
DEV float range_weight(float dg, const WeightParams& wp) {
  if (KIND == 0) return __builtin_amdgcn_exp2f(-(dg * dg) * wp.range_c2);
  const float ad = fabsf(dg);
  if (ad >= kSentinelGap) return 0.0f;
  float pw;
  if (wp.alpha_r == 0.0f) pw = 1.0f;
  else pw = ad > 0.0f ? __builtin_amdgcn_exp2f(wp.alpha_r * __builtin_amdgcn_logf(ad)) : 0.0f;
  return __builtin_amdgcn_rcpf(pw + wp.eps);
}

DEV float recip(float x) { return __builtin_amdgcn_rcpf(x); }
DEV double recip(double x) { return 1.0 / x; }

// Element m of a chunk (local index; negative = the previous chunk's tail)
// lies in chunk row floor(m / (2r+1)) at position q = m mod (2r+1).  Chunks
// start on even subsystem rows (R is even), so a row's parity is that of its
// local row index: even rows run k-r..k+r, odd rows k+r..k-r (Sec. 2.1 with
// 1-based rows, where the even ones are reversed).
template <int r>
DEV constexpr int row_of(int m) {
  return m >= 0 ? m / (2 * r + 1) : -1 - ((-m - 1) / (2 * r + 1));
}
template <int r>
DEV constexpr int col_of(int m) {  // offset from the centre column k
  return (row_of<r>(m) & 1) ? (r - (m - row_of<r>(m) * (2 * r + 1)))
                            : ((m - row_of<r>(m) * (2 * r + 1)) - r);
}

// Small dense helpers on r x r blocks.  chol leaves a factor that chol_solve
// applies: the Cholesky factor for n > 1 with the reciprocals of its
// diagonal entries on the diagonal (one division per entry; the solves then
// multiply); for n = 1 the reciprocal of the scalar itself (one rcp instead
// of a square root and two divisions).
template <int n, typename Acc>
DEV void chol(Acc (&A)[n][n]) {
  if constexpr (n == 1) {
    A[0][0] = recip(A[0][0]);
    return;
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    Acc d = A[j][j];
#pragma unroll
    for (int t = 0; t < j; ++t) d -= A[j][t] * A[j][t];
    const Acc inv = Acc(1) / sqrt(d);
    A[j][j] = inv;
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      Acc v = A[i][j];
#pragma unroll
      for (int t = 0; t < j; ++t) v -= A[i][t] * A[j][t];
      A[i][j] = v * inv;
    }
  }
}

template <int n, int m, typename Acc>
DEV void chol_solve(const Acc (&Lc)[n][n], Acc (&B)[n][m]) {
  if constexpr (n == 1) {
#pragma unroll
    for (int c = 0; c < m; ++c) B[0][c] *= Lc[0][0];
    return;
  }
#pragma unroll
  for (int c = 0; c < m; ++c) {
#pragma unroll
    for (int i = 0; i < n; ++i) {
      Acc v = B[i][c];
#pragma unroll
      for (int t = 0; t < i; ++t) v -= Lc[i][t] * B[t][c];
      B[i][c] = v * Lc[i][i];
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
      Acc v = B[i][c];
#pragma unroll
      for (int t = i + 1; t < n; ++t) v -= Lc[t][i] * B[t][c];
      B[i][c] = v * Lc[i][i];
    }
  }
}

// Inverse of a small SPD matrix through its Cholesky factor.
template <int n, typename Acc>
DEV void spd_inverse(const Acc (&A)[n][n], Acc (&Ai)[n][n]) {
  if constexpr (n == 1) {
    Ai[0][0] = recip(A[0][0]);
    return;
  }
  Acc Lc[n][n];
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) Lc[i][j] = A[i][j];
  chol<n, Acc>(Lc);
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) Ai[i][j] = (i == j) ? Acc(1) : Acc(0);
  chol_solve<n, n, Acc>(Lc, Ai);
}

// C = A * B (n x k times k x m), C must not alias.
template <int n, int k, int m, typename Acc>
DEV void mm(const Acc (&A)[n][k], const Acc (&B)[k][m], Acc (&C)[n][m]) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) {
      Acc v = Acc(0);
#pragma unroll
      for (int t = 0; t < k; ++t) v += A[i][t] * B[t][j];
      C[i][j] = v;
    }
}

// C -= A^T * B.
template <int n, int k, int m, typename Acc>
DEV void sub_AtB(const Acc (&A)[k][n], const Acc (&B)[k][m], Acc (&C)[n][m]) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) {
      Acc v = C[i][j];
#pragma unroll
      for (int t = 0; t < k; ++t) v -= A[t][i] * B[t][j];
      C[i][j] = v;
    }
}

template <int n, int m, typename Acc>
DEV void shfl_up_blk(const Acc (&src)[n][m], Acc (&dst)[n][m], int delta, int lane) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) {
      const Acc v = __shfl_up(src[i][j], delta, kWave);
      dst[i][j] = lane >= delta ? v : Acc(0);
    }
}

template <int n, int m, typename Acc>
DEV void shfl_down_blk(const Acc (&src)[n][m], Acc (&dst)[n][m], int delta, int lane) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) {
      const Acc v = __shfl_down(src[i][j], delta, kWave);
      dst[i][j] = lane + delta < kWave ? v : Acc(0);
    }
}

// ---------------------------------------------------------------------------
// Layout of the per-chunk Schur complement contributions written by k_reduce
// (strip-major: sum[(ki * P + j) * F + f]).
template <int r, int CB>
struct IfaceLayout {
  static constexpr int T2 = r * (r + 1) / 2;
  static constexpr int oW = 0;                  // A_SS - A_SI A_I^-1 A_IS of S_j (lower)
  static constexpr int oRf = T2;                // f_S - A_SI A_I^-1 f_I of S_j
  static constexpr int oTT = T2 + r * CB;       // A_TI A_I^-1 A_IT of T = S_{j-1} (lower)
  static constexpr int oRT = 2 * T2 + r * CB;   // A_TI A_I^-1 f_I
  static constexpr int oTB = 2 * T2 + 2 * r * CB;  // S_j <-> S_{j-1} coupling after elimination
  static constexpr int F = 2 * T2 + 2 * r * CB + r * r;
};

// lambda of the pass: the device override when given, else the host value
// (validated on the host).  A negative device value is clamped to 0, where
// A_s = I + lambda L stops being positive definite; NaN passes through.
DEV float load_lambda(const float* lam_dev, float lam_host) {
  if (!lam_dev) return lam_host;
  const float v = *lam_dev;
  return v < 0.0f ? 0.0f : v;
}

DEV int centre_of(int ki, const PassGeom& geo, int r) {
  return min(r + ki * geo.stride, geo.W - 1 - r);
}

// Number of strip centres whose 2r+1 columns cover column b.
DEV int cover_count(int b, const PassGeom& geo, int r) {
  const int lo = max(r, b - r), hi = min(geo.W - 1 - r, b + r);
  const int t = geo.stride;
  const int first = (lo - r + t - 1) / t, last = (hi - r) / t;
  int c = max(0, last - first + 1);
  const int span = geo.W - 1 - 2 * r;
  if (span % t != 0 && geo.W - 1 - r >= lo && geo.W - 1 - r <= hi) c += 1;
  return c;
}


// ---------------------------------------------------------------------------
// Source planes of a tile: NX channels of X, then channels of X2, both from
// channel c0 on (`plane` floats apart).  The forward kernels read X only; the
// backward ones read the saved pass input (X) and the output gradient (X2).
template <int NX>
struct PlaneSrc {
  const float* X;
  const float* X2;
  int c0, plane;
  DEV const float* at(int p) const {
    return p < NX ? X + (c0 + p) * plane : X2 + (c0 + p - NX) * plane;
  }
};

// LDS tile of a block: rows a in [a_lo - 1, a_lo + Q*R + 1) of the pass, columns
// b in [colbase, colbase + TB), planes: guidance then NP image planes.  Rows
// or columns outside the image hold 0 (never used as pixels).  Loads are
// issued in batches of BATCH per thread before any LDS store, so one memory
// latency covers the batch; consecutive threads read consecutive addresses
// (b in the column pass, a in the row pass).
template <int NP, int NX, int TA, int NT, int BATCH>
DEV void load_tile(float* lds, const float* __restrict__ G, const PlaneSrc<NX>& src,
                   const PassGeom& geo, int a_lo, int colbase, int TB, int pitch, int tid) {
  const int total = TA * TB;
  const bool colpass = geo.sb == 1;
  for (int base = 0; base < total; base += NT * BATCH) {
    float v[NP + 1][BATCH];
    int dst[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int idx = base + u * NT + tid;
      int ta, tb;
      if (colpass) {
        ta = idx / TB;
        tb = idx - ta * TB;
      } else {
        tb = idx / TA;
        ta = idx - tb * TA;
      }
      const int a = a_lo - 1 + ta, b = colbase + tb;
      const bool rowok = a >= 0 && a < geo.L;
      const bool in = idx < total && rowok && b < geo.W;
      const int o = in ? (colpass ? a * (int)geo.sa + b : a + b * (int)geo.sb) : 0;
      dst[u] = idx < total ? ta * pitch + tb : -1;
      const float gv = G[o];
      // Rows outside the subsystem hold a sentinel guidance value: every edge
      // to them gets weight 0 (see range_weight).
      v[0][u] = in ? gv : (rowok ? 0.0f : kSentinel);
#pragma unroll
      for (int p = 1; p <= NP; ++p) {
        const float xv = src.at(p - 1)[o];
        v[p][u] = in ? xv : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u)
      if (dst[u] >= 0) {
#pragma unroll
        for (int p = 0; p <= NP; ++p) lds[p * TA * pitch + dst[u]] = v[p][u];
      }
  }
}


// Stride-1 tiles (TB = 64 + 2r columns), loaded with wave-uniform row or
// column bases so that every load is a uniform pointer plus a fixed lane
// offset.  Column pass: wave wq loads tile rows wq, wq+Q, ... (contiguous in
// memory), lane l columns l and l+64.  Row pass: wave wq loads tile columns
// wq, wq+Q, ... (contiguous along a), lane l rows l and l+64.  All loads of a
// thread are issued before its LDS stores.
template <int r, int NP, int NX, int TA, int Q>
DEV void load_tile_s1(float* lds, const float* __restrict__ G, const PlaneSrc<NX>& src,
                      const PassGeom& geo, int a_lo, int colbase, int pitch, int lane, int wq) {
  constexpr int TB = kWave + 2 * r;
  if (geo.sb == 1) {
    constexpr int NR = (TA + Q - 1) / Q, NH = (TB + kWave - 1) / kWave;
    const int sa = (int)geo.sa;
    int lo[NH];
    bool lv[NH], cok[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int tb = lane + kWave * h, b = colbase + tb;
      lv[h] = tb < TB;
      cok[h] = lv[h] && b < geo.W;
      lo[h] = cok[h] ? b : colbase;
    }
    float v[NR][NH][NP + 1];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int ta = wq + i * Q, a = a_lo - 1 + ta;
      if (ta < TA && a >= 0 && a < geo.L) {
        const float* gr = G + a * sa;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          v[i][h][0] = gr[lo[h]];
#pragma unroll
          for (int c = 0; c < NP; ++c) v[i][h][c + 1] = (src.at(c) + a * sa)[lo[h]];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int ta = wq + i * Q, a = a_lo - 1 + ta;
      if (ta < TA) {
        const bool rowok = a >= 0 && a < geo.L;
#pragma unroll
        for (int h = 0; h < NH; ++h)
          if (lv[h]) {
            float* d = lds + ta * pitch + lane + kWave * h;
            d[0] = rowok ? (cok[h] ? v[i][h][0] : 0.0f) : kSentinel;
#pragma unroll
            for (int c = 0; c < NP; ++c) d[(c + 1) * TA * pitch] = (rowok && cok[h]) ? v[i][h][c + 1] : 0.0f;
          }
      }
    }
  } else {
    constexpr int NC = (TB + Q - 1) / Q, NH = (TA + kWave - 1) / kWave;
    const int sb = (int)geo.sb;
    int lo[NH];
    bool lv[NH], aok[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int ta = lane + kWave * h, a = a_lo - 1 + ta;
      lv[h] = ta < TA;
      aok[h] = lv[h] && a >= 0 && a < geo.L;
      lo[h] = aok[h] ? a : 0;
    }
    float v[NC][NH][NP + 1];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int tb = wq + i * Q, b = colbase + tb;
      if (tb < TB && b < geo.W) {
        const float* gc = G + b * sb;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          v[i][h][0] = gc[lo[h]];
#pragma unroll
          for (int c = 0; c < NP; ++c) v[i][h][c + 1] = (src.at(c) + b * sb)[lo[h]];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int tb = wq + i * Q, b = colbase + tb;
      if (tb < TB) {
        const bool bok = b < geo.W;
#pragma unroll
        for (int h = 0; h < NH; ++h)
          if (lv[h]) {
            float* d = lds + (lane + kWave * h) * pitch + tb;
            d[0] = aok[h] ? (bok ? v[i][h][0] : 0.0f) : kSentinel;
#pragma unroll
            for (int c = 0; c < NP; ++c) d[(c + 1) * TA * pitch] = (aok[h] && bok) ? v[i][h][c + 1] : 0.0f;
          }
      }
    }
  }
}

// v shifted up by one lane across the wave (lane 0 receives 0).
DEV float lane_shr1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x138, 0xf, 0xf, false));
}

// The chunk of one lane: element values come from the LDS tile.
template <int r, int R, bool S1>
struct ChunkView {
  static constexpr int w = 2 * r + 1;
  static constexpr int E = R * w;
  static constexpr int PITCH1 = kWave + 2 * r + 1;   // pitch of stride-1 tiles
  static_assert(R >= 2 && R % 2 == 0, "chunks must start on even rows");
  const float* base;   // plane 0 at (tile row of the chunk's first row, column k)
  int pitch, plane, a0, L;
  DEV int off(int m) const {
    const int p = S1 ? PITCH1 : pitch;
    return row_of<r>(m) * p + col_of<r>(m);
  }
  DEV bool ok(int m) const {
    const int a = a0 + row_of<r>(m);
    return a >= 0 && a < L;
  }
  DEV float g(int m) const { return base[off(m)]; }
  DEV float f(int m, int c) const { return base[(c + 1) * plane + off(m)]; }
};

// The chunk of one lane read straight from global memory (column pass at
// stride 1, where the 64 lanes of a wave are 64 adjacent columns, so every
// element load is one coalesced row segment): no LDS tile and no workgroup
// barrier, so the waves of a SIMD drift apart and overlap their loads with
// each other's arithmetic.  Buffer descriptors cover exactly the image rows
// the chunk touches (its rows and one row on each side), so offsets are
// 32-bit and rows outside the image read 0; the guidance of those rows is
// replaced by the sentinel.
template <int r, int R, int NP>
struct GlobalChunk {
  static constexpr int w = 2 * r + 1;
  static constexpr int E = R * w;
  __amdgpu_buffer_rsrc_t rg, rf[NP];
  int lane_off;   // byte offset of (row a0, column k - r) from the descriptor base
  int row_bytes, a0, L;
  template <int NX>
  DEV void init(const float* G, const PlaneSrc<NX>& src, const PassGeom& geo, int a0_, int k) {
    a0 = a0_;
    L = geo.L;
    const int n = (int)geo.sa;
    const int lo = max(a0 - 1, 0), hi = min(a0 + R + 1, L);
    const int base = lo * n, bytes = (hi - lo) * n * 4;
    rg = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(G + base), (short)0, bytes, 0x00020000);
#pragma unroll
    for (int p = 0; p < NP; ++p)
      rf[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(src.at(p) + base), (short)0, bytes,
                                                0x00020000);
    row_bytes = n * 4;
    lane_off = ((a0 - lo) * n + k - r) * 4;
  }
  DEV int off(int m) const { return lane_off + row_of<r>(m) * row_bytes + (col_of<r>(m) + r) * 4; }
  DEV bool ok(int m) const {
    const int a = a0 + row_of<r>(m);
    return a >= 0 && a < L;
  }
  DEV float g(int m) const {
    const float v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, off(m), 0, 0));
    return ok(m) ? v : kSentinel;
  }
  DEV float f(int m, int c) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rf[c], off(m), 0, 0));
  }
};

// lambda * w(m, m+d) for local m in [-r, E) and d = 1..r, at lw[m + r][d - 1].
// Ends outside the subsystem read the sentinel guidance, so their edges
// weigh 0 and the padding elements are decoupled from the subsystem.
template <int r, int KIND, class V>
DEV void chunk_weights(const V& cv, const WeightParams& wp, const float (&lamS)[r + 1],
                       float (&lw)[V::E + r][r]) {
  constexpr int E = V::E;
  float gv[E + 2 * r];
#pragma unroll
  for (int m = -r; m < E + r; ++m) gv[m + r] = cv.g(m);
#pragma unroll
  for (int m = -r; m < E; ++m) {
#pragma unroll
    for (int d = 1; d <= r; ++d) {
      lw[m + r][d - 1] = lamS[d] * range_weight<KIND>(gv[m + r] - gv[m + d + r], wp);
    }
  }
}

// Diagonal of A_s at local element m: 1 + lambda * (sum of its edge weights).
template <int r, int E, typename Acc>
DEV Acc diag_at(const float (&lw)[E + r][r], int m) {
  Acc s = Acc(1);
#pragma unroll
  for (int d = 1; d <= r; ++d) s += Acc(lw[m + r][d - 1]) + Acc(lw[m - d + r][d - 1]);
  return s;
}

template <int r>
DEV int tile_width(int stride) { return stride == 1 ? kWave + 2 * r : (kWave - 1) * stride + 2 * r + 1; }

// Reciprocal cover counts of the 2r+1 columns k-r..k+r of strip k: the
// adjoint of the averaging of Sec. 2.3 divides the output gradient by them.
template <int r, bool S1>
DEV void inv_counts(int k, const PassGeom& geo, float (&ic)[2 * r + 1]) {
#pragma unroll
  for (int q = 0; q <= 2 * r; ++q) {
    const int b = k - r + q;
    const int c = S1 ? min(geo.W - 1 - r, b + r) - max(r, b - r) + 1 : cover_count(b, geo, r);
    ic[q] = 1.0f / float(max(c, 1));
  }
}

// First strip of expand block bx (blocks own OW pass columns each; the strips
// of a block are those whose columns touch the columns it owns).
DEV int expand_first_strip(int bx, int OW, const PassGeom& geo, int r) {
  const int b_lo = bx * OW;
  int ki;
  if (geo.stride == 1) {
    ki = max(0, b_lo - 2 * r);
  } else {
    const int t = b_lo - 2 * r;
    ki = t <= 0 ? 0 : (t + geo.stride - 1) / geo.stride;
  }
  return min(ki, geo.nK - 1);
}

// Loads and stores of interface data.  COH: the data passes between
// workgroups of one launch (possibly on different XCDs, whose L2 caches are
// not coherent with each other), so it is written through to and read from
// the device-coherent level (agent-scope relaxed atomic accesses, one word
// each); otherwise plain accesses (the data crosses a kernel boundary).
template <bool COH, typename T>
DEV T ld_if(const T* p) {
  if constexpr (COH) return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool COH, typename T>
DEV void st_if(T* p, T v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// Guidance of the chunk elements m in [-r, E + r) (gv[m + r]) and the weights
// omega(m, m+d) of Eq. (2) without lambda (om[m + r][d - 1], m in [-r, E)).
template <int r, int KIND, class V>
DEV void chunk_omega(const V& cv, const WeightParams& wp, float (&gv)[V::E + 2 * r],
                     float (&om)[V::E + r][r]) {
  constexpr int E = V::E;
#pragma unroll
  for (int m = -r; m < E + r; ++m) gv[m + r] = cv.g(m);
#pragma unroll
  for (int m = -r; m < E; ++m)
#pragma unroll
    for (int d = 1; d <= r; ++d)
      om[m + r][d - 1] = wp.spatial[d] * range_weight<KIND>(gv[m + r] - gv[m + d + r], wp);
}

// d omega / d dG for dG = G_p - G_q, given omega.  exp: -omega dG / sigma_r^2.
// frac: -omega alpha_r |dG|^alpha_r / (dG (|dG|^alpha_r + eps)), taken as 0 at
// dG = 0 where it is not differentiable for alpha_r <= 1.  The factor
// |dG|^a / (|dG|^a + eps) is formed as 1 / (1 + eps / |dG|^a): |dG|^a
// overflows float32 for the sentinel guidance of rows outside the image once
// alpha_r > 38.5 / 30, and the other form would then be inf * 0.
template <int KIND>
DEV float domega(float w, float dg, const WeightParams& wp) {
  if (KIND == 0) return -w * dg * wp.inv_sr2;
  const float ad = fabsf(dg);
  if (!(ad > 0.0f) || wp.alpha_r == 0.0f) return 0.0f;
  const float pw = __builtin_amdgcn_exp2f(wp.alpha_r * __builtin_amdgcn_logf(ad));
  const float share = __builtin_amdgcn_rcpf(1.0f + wp.eps * __builtin_amdgcn_rcpf(pw));
  return -w * wp.alpha_r * share / dg;
}

// ---------------------------------------------------------------------------
// k_reduce: Schur complement contributions of every chunk of 64 strips.
// Forward: the right-hand sides are the CB channels of X.  Backward: also the
// CB channels of the output gradient X2 divided by the cover counts, so the
// pass solution and the adjoint solve share one elimination (NR = 2 CB).
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE,
          bool DIRECT = false, bool COH = false>
DEV void reduce_tile(const PassGeom& geo, const WeightParams& wp, float lam, int pch,
                     Acc* __restrict__ sum, int bx, int by, float* smem,
                     const float* G = nullptr, const PlaneSrc<CB>* src = nullptr);

// Block (bx, by) of the reduce grid: strips [64 bx, 64 bx + 64), chunks
// [Q by, Q by + Q).  smem: the block's dynamic LDS.
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE>
DEV void reduce_block(const float* __restrict__ X, const float* __restrict__ X2,
                      const float* __restrict__ G, const PassGeom& geo, const WeightParams& wp,
                      float lam, int c0, int pitch, Acc* __restrict__ sum, int bx, int by,
                      float* smem) {
  constexpr int NR = MODE == kModeBackward ? 2 * CB : CB;
  using CV = ChunkView<r, R, S1>;
  constexpr int TA = Q * R + 2;
  const int lane = threadIdx.x % kWave;
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int ki_lo = bx * kWave;
  const int a_lo = by * Q * R;
  const int colbase = centre_of(ki_lo, geo, r) - r;
  const int TB = S1 ? kWave + 2 * r : tile_width<r>(geo.stride);
  const int pch = S1 ? CV::PITCH1 : pitch;
  const PlaneSrc<CB> src{X, X2, c0, (int)geo.plane};
  if constexpr (S1)
    load_tile_s1<r, NR, CB, TA, Q>(smem, G, src, geo, a_lo, colbase, pch, lane, wq);
  else
    load_tile<NR, CB, TA, kWave * Q, 8>(smem, G, src, geo, a_lo, colbase, TB, pch, threadIdx.x);
  __syncthreads();
  reduce_tile<r, CB, R, Q, S1, KIND, Acc, MODE>(geo, wp, lam, pch, sum, bx, by, smem);
}

// The elimination of a block whose tile is in LDS (see reduce_block), or, with
// DIRECT, whose chunks are read from global memory (stride-1 column pass).
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE, bool DIRECT,
          bool COH>
DEV void reduce_tile(const PassGeom& geo, const WeightParams& wp, float lam, int pch,
                     Acc* __restrict__ sum, int bx, int by, float* smem, const float* G,
                     const PlaneSrc<CB>* src) {
  constexpr int NR = MODE == kModeBackward ? 2 * CB : CB;
  using CV = ChunkView<r, R, S1>;
  using LY = IfaceLayout<r, NR>;
  constexpr int E = CV::E;
  constexpr int TA = Q * R + 2;
  const int lane = threadIdx.x % kWave;
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int ki_lo = bx * kWave;
  const int j0 = by * Q, j = j0 + wq;
  const int colbase = centre_of(ki_lo, geo, r) - r;
  const int ki = ki_lo + lane;
  const bool active = ki < geo.nK && j < geo.P;
  const bool hasT = j > 0, hasB = j + 1 < geo.P;
  Acc W[r + 1][r + 1];   // Schur complement on the window, lower triangle
  Acc Bt[r + 1][r];      // window couplings to the previous separator
  Acc Rw[r + 1][NR];     // window right-hand sides
  Acc TT[r][r], RT[r][NR];
  if (active) {
    float lamS[r + 1];
#pragma unroll
    for (int d = 0; d <= r; ++d) lamS[d] = lam * wp.spatial[d];
    const int k = centre_of(ki, geo, r);
    typename std::conditional<DIRECT, GlobalChunk<r, R, NR>, CV>::type cv;
    if constexpr (DIRECT) {
      cv.init(G, *src, geo, j * R, k);
    } else {
      cv.base = smem + (wq * R + 1) * pch + (k - colbase);
      cv.pitch = pch;
      cv.plane = TA * pch;
      cv.a0 = j * R;
      cv.L = geo.L;
    }
    // Direct reads: every chunk value is requested before the elimination
    // starts, so the loads are in flight together instead of inside the chain.
    float fpre[DIRECT ? E : 1][NR];
    if constexpr (DIRECT) {
#pragma unroll
      for (int m = 0; m < E; ++m)
#pragma unroll
        for (int c = 0; c < NR; ++c) fpre[m][c] = cv.f(m, c);
    }
    float lw[E + r][r];
    chunk_weights<r, KIND>(cv, wp, lamS, lw);
    float ic[2 * r + 1];
    if constexpr (MODE != kModeForward) inv_counts<r, S1>(k, geo, ic);
    auto fval = [&](int m, int c) -> Acc {   // 0 outside the subsystem
      const float v = DIRECT ? fpre[DIRECT ? m : 0][c] : cv.f(m, c);
      if ((MODE == kModeBackward && c >= CB) || MODE == kModeAdjoint)
        return Acc(v * ic[col_of<r>(m) + r]);
      return Acc(v);
    };
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int b = 0; b < r; ++b) TT[a][b] = Acc(0);
#pragma unroll
      for (int c = 0; c < NR; ++c) RT[a][c] = Acc(0);
    }
#pragma unroll
    for (int a = 0; a < r; ++a) {
      W[a][a] = diag_at<r, E, Acc>(lw, a);
#pragma unroll
      for (int b = 0; b < a; ++b) W[a][b] = -Acc(lw[b + r][a - b - 1]);
#pragma unroll
      for (int c = 0; c < r; ++c) Bt[a][c] = (c >= a) ? -Acc(lw[c][a + r - c - 1]) : Acc(0);
#pragma unroll
      for (int c = 0; c < NR; ++c) Rw[a][c] = fval(a, c);
    }
    auto step = [&](const int m) {
      const int n = m + r;   // element entering the window
      if (n < E) {
        W[r][r] = diag_at<r, E, Acc>(lw, n);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = -Acc(lw[m + b + r][r - b - 1]);
#pragma unroll
        for (int c = 0; c < NR; ++c) Rw[r][c] = fval(n, c);
      } else {               // past the end of the subsystem
        W[r][r] = Acc(1);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = Acc(0);
#pragma unroll
        for (int c = 0; c < NR; ++c) Rw[r][c] = Acc(0);
      }
#pragma unroll
      for (int c = 0; c < r; ++c) Bt[r][c] = Acc(0);
      const Acc invD = recip(W[0][0]);
      Acc l[r + 1];
#pragma unroll
      for (int a = 1; a <= r; ++a) l[a] = W[a][0] * invD;
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int b = 1; b <= a; ++b) W[a][b] -= l[a] * W[b][0];
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Bt[a][c] -= l[a] * Bt[0][c];
#pragma unroll
      for (int c = 0; c < r; ++c) {
        const Acc bs = Bt[0][c] * invD;
#pragma unroll
        for (int c2 = 0; c2 <= c; ++c2) TT[c][c2] += bs * Bt[0][c2];
#pragma unroll
        for (int h = 0; h < NR; ++h) RT[c][h] += bs * Rw[0][h];
      }
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[a][h] -= l[a] * Rw[0][h];
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) W[a][b] = W[a + 1][b + 1];
#pragma unroll
        for (int c = 0; c < r; ++c) Bt[a][c] = Bt[a + 1][c];
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[a][h] = Rw[a + 1][h];
      }
    };
    // Interior of a chunk with a separator: elements 0..E-r-1.  The last chunk
    // has no separator and eliminates all E (padding past the end is inert).
#pragma unroll
    for (int m = 0; m < E - r; ++m) step(m);
    if (!hasB) {
#pragma unroll
      for (int m = E - r; m < E; ++m) step(m);
    }
  }
  __syncthreads();   // tile reads done: the LDS now stages the block's output

  Acc* st = reinterpret_cast<Acc*>(smem) + (lane * Q + wq) * LY::F;
  if (active) {
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        st[LY::oW + t] = hasB ? W[a][b] : Acc(0);
        st[LY::oTT + t] = hasT ? TT[a][b] : Acc(0);
        ++t;
      }
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        st[LY::oRf + a * NR + h] = hasB ? Rw[a][h] : Acc(0);
        st[LY::oRT + a * NR + h] = hasT ? RT[a][h] : Acc(0);
      }
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) st[LY::oTB + a * r + c] = (hasT && hasB) ? Bt[a][c] : Acc(0);
  }
  __syncthreads();
  // strip-major output: Q*F consecutive values per strip
  const int qv = min(Q, geo.P - j0);
  const Acc* stg = reinterpret_cast<const Acc*>(smem);
  for (int idx = threadIdx.x; idx < kWave * Q * LY::F; idx += kWave * Q) {
    const int s = idx / (Q * LY::F), t = idx - s * (Q * LY::F);
    if (ki_lo + s < geo.nK && t < qv * LY::F)
      st_if<COH>(sum + ((size_t)(ki_lo + s) * geo.P + j0) * LY::F + t, stg[idx]);
  }
}

template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE>
__global__ __launch_bounds__(kWave* Q) void k_reduce(
    const float* __restrict__ X, const float* __restrict__ X2, const float* __restrict__ G,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    int pitch, Acc* __restrict__ sum) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  reduce_block<r, CB, R, Q, S1, KIND, Acc, MODE>(
      zmove(X, geo.zx, z), zmove(X2, geo.zx2, z), zmove(G, geo.zg, z), geo,
      wp, load_lambda(lam_dev, lam_host), c0, pitch, zmove_bytes(sum, geo.zi, z), blockIdx.x,
      blockIdx.y, smem);
}

// ---------------------------------------------------------------------------
// Separator system of one strip: Sigma_jj = W_j - TT_{j+1},
// Sigma_{j,j+1}[a][c] = TB_{j+1}[c][a], rhs_j = Rf_j - RT_{j+1}, j = 0..P-2.
template <int r, int CB, typename Acc, bool COH = false>
struct SepReader {
  using LY = IfaceLayout<r, CB>;
  const Acc* S;   // this strip's contributions
  int P;
  DEV Acc at(int j, int f) const { return ld_if<COH>(S + (size_t)j * LY::F + f); }
  DEV void diag(int j, Acc (&A)[r][r]) const {
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        A[a][b] = at(j, LY::oW + t) - at(j + 1, LY::oTT + t);
        A[b][a] = A[a][b];
        ++t;
      }
  }
  DEV void rhs(int j, Acc (&y)[r][CB]) const {
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h)
        y[a][h] = at(j, LY::oRf + a * CB + h) - at(j + 1, LY::oRT + a * CB + h);
  }
  DEV void off(int j, Acc (&U)[r][r]) const {   // Sigma_{j,j+1}; zero past the last
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) U[a][c] = (j + 1 < P - 1) ? at(j + 1, LY::oTB + c * r + a) : Acc(0);
  }
};

// SepReader over records prefetched into registers: chunks s .. s + nrec - 1
// of one strip (indices past the last chunk read the last one), loaded
// together before the elimination so that their latency is paid once.
// Calls index chunks absolutely; the indices are s plus compile-time offsets.
template <int r, int CB, int NREC, typename Acc, bool COH = false>
struct PreReader {
  using LY = IfaceLayout<r, CB>;
  Acc rec[NREC][LY::F];
  int s, P;
  DEV void load(const Acc* __restrict__ S, int s_, int P_, int nrec) {
    s = s_;
    P = P_;
#pragma unroll
    for (int i = 0; i < NREC; ++i) {
      if (i < nrec) {
        const int jj = min(s + i, P - 1);
#pragma unroll
        for (int f = 0; f < LY::F; ++f) rec[i][f] = ld_if<COH>(S + (size_t)jj * LY::F + f);
      }
    }
  }
  DEV Acc at(int j, int f) const { return rec[j - s][f]; }
  DEV void diag(int j, Acc (&A)[r][r]) const {
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        A[a][b] = at(j, LY::oW + t) - at(j + 1, LY::oTT + t);
        A[b][a] = A[a][b];
        ++t;
      }
  }
  DEV void rhs(int j, Acc (&y)[r][CB]) const {
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h)
        y[a][h] = at(j, LY::oRf + a * CB + h) - at(j + 1, LY::oRT + a * CB + h);
  }
  DEV void off(int j, Acc (&U)[r][r]) const {
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) U[a][c] = (j + 1 < P - 1) ? at(j + 1, LY::oTB + c * r + a) : Acc(0);
  }
};

// The reduced system of one strip's separators after each lane eliminated
// its own run (lane l keeps the last block of its run): block cyclic
// reduction across the 64 lanes, then each lane's solution X and the one of
// the lane before it (XT, zero on lane 0).
template <int r, int CB, typename Acc>
DEV void iface_pcr_levels(const Acc (&S)[r][r], const Acc (&Bt)[r][r], const Acc (&Rr)[r][CB],
                          const Acc (&TT)[r][r], const Acc (&RT)[r][CB], bool active, int m,
                          int n, int lane, Acc (&X)[r][CB], Acc (&XT)[r][CB]) {
  // PCR level: lane l's unknown X_l = x_{e-1}:
  //   A_l X_{l-1} + B_l X_l + C_l X_{l+1} = d_l with
  //   A_l = Bt_l, B_l = S_l - TT_{l+1}, C_l = Bt_{l+1}^T, d_l = R_l - RT_{l+1}.
  Acc A[r][r], B[r][r], Cc[r][r], d[r][CB];
  {
    Acc TTn[r][r], RTn[r][CB], Btn[r][r];
    shfl_down_blk<r, r, Acc>(TT, TTn, 1, lane);
    shfl_down_blk<r, CB, Acc>(RT, RTn, 1, lane);
    shfl_down_blk<r, r, Acc>(Bt, Btn, 1, lane);
    const bool nextActive = (lane + 1) * m < n;
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        A[a][c] = active ? Bt[a][c] : Acc(0);
        B[a][c] = active ? S[a][c] - (nextActive ? TTn[a][c] : Acc(0)) : (a == c ? Acc(1) : Acc(0));
        Cc[a][c] = (active && nextActive) ? Btn[c][a] : Acc(0);
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) d[a][h] = active ? Rr[a][h] - (nextActive ? RTn[a][h] : Acc(0)) : Acc(0);
    }
  }
#pragma unroll
  for (int delta = 1; delta < kWave; delta *= 2) {
    Acc Bi[r][r];
    spd_inverse<r, Acc>(B, Bi);
    Acc Bim[r][r], Am[r][r], Cm[r][r], dm[r][CB];
    Acc Bip[r][r], Ap[r][r], Cp[r][r], dp[r][CB];
    shfl_up_blk<r, r, Acc>(Bi, Bim, delta, lane);
    shfl_up_blk<r, r, Acc>(A, Am, delta, lane);
    shfl_up_blk<r, r, Acc>(Cc, Cm, delta, lane);
    shfl_up_blk<r, CB, Acc>(d, dm, delta, lane);
    shfl_down_blk<r, r, Acc>(Bi, Bip, delta, lane);
    shfl_down_blk<r, r, Acc>(A, Ap, delta, lane);
    shfl_down_blk<r, r, Acc>(Cc, Cp, delta, lane);
    shfl_down_blk<r, CB, Acc>(d, dp, delta, lane);
    Acc al[r][r], ga[r][r];
    mm<r, r, r, Acc>(A, Bim, al);
    mm<r, r, r, Acc>(Cc, Bip, ga);
    Acc An[r][r], Cn[r][r], t1[r][r], t2[r][r], e1[r][CB], e2[r][CB];
    mm<r, r, r, Acc>(al, Am, An);
    mm<r, r, r, Acc>(ga, Cp, Cn);
    mm<r, r, r, Acc>(al, Cm, t1);
    mm<r, r, r, Acc>(ga, Ap, t2);
    mm<r, r, CB, Acc>(al, dm, e1);
    mm<r, r, CB, Acc>(ga, dp, e2);
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        A[a][c] = -An[a][c];
        Cc[a][c] = -Cn[a][c];
        B[a][c] = B[a][c] - t1[a][c] - t2[a][c];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) d[a][h] = d[a][h] - e1[a][h] - e2[a][h];
    }
  }
  {
    Acc Bc[r][r];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) Bc[a][c] = B[a][c];
    chol<r, Acc>(Bc);
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) X[a][h] = d[a][h];
    chol_solve<r, CB, Acc>(Bc, X);
  }
  shfl_up_blk<r, CB, Acc>(X, XT, 1, lane);
}

// Block exchanges between the NL lanes of a workgroup (NL = 64 x waves)
// through LDS: value f of lane L at xs[f * NL + L].
template <int n, int m, int NL, typename Acc>
DEV void lds_put(Acc* xs, int f0, const Acc (&b)[n][m], int L) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) xs[(f0 + i * m + j) * NL + L] = b[i][j];
}
// b = the block of lane src, or 0 where !ok.
template <int n, int m, int NL, typename Acc>
DEV void lds_get(const Acc* xs, int f0, Acc (&b)[n][m], int src, bool ok) {
  const int s = ok ? src : 0;
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) {
      const Acc v = xs[(f0 + i * m + j) * NL + s];
      b[i][j] = ok ? v : Acc(0);
    }
}

// iface_pcr_levels over the NL lanes of a workgroup: the same reduced system
// and block cyclic reduction (log2 NL levels), with every neighbour exchange
// through LDS (xs: NL x (3 r^2 + r CB) values).  Called by all NL threads.
template <int r, int CB, typename Acc, int NL>
DEV void iface_pcr_levels_mw(const Acc (&S)[r][r], const Acc (&Bt)[r][r], const Acc (&Rr)[r][CB],
                             const Acc (&TT)[r][r], const Acc (&RT)[r][CB], bool active, int m,
                             int n, int L, Acc* xs, Acc (&X)[r][CB], Acc (&XT)[r][CB]) {
  constexpr int RR = r * r, RC = r * CB;
  Acc A[r][r], B[r][r], Cc[r][r], d[r][CB];
  {
    Acc TTn[r][r], RTn[r][CB], Btn[r][r];
    lds_put<r, r, NL>(xs, 0, TT, L);
    lds_put<r, CB, NL>(xs, RR, RT, L);
    lds_put<r, r, NL>(xs, RR + RC, Bt, L);
    __syncthreads();
    const bool has = L + 1 < NL;
    lds_get<r, r, NL>(xs, 0, TTn, L + 1, has);
    lds_get<r, CB, NL>(xs, RR, RTn, L + 1, has);
    lds_get<r, r, NL>(xs, RR + RC, Btn, L + 1, has);
    __syncthreads();
    const bool nextActive = (L + 1) * m < n;
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        A[a][c] = active ? Bt[a][c] : Acc(0);
        B[a][c] = active ? S[a][c] - (nextActive ? TTn[a][c] : Acc(0)) : (a == c ? Acc(1) : Acc(0));
        Cc[a][c] = (active && nextActive) ? Btn[c][a] : Acc(0);
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) d[a][h] = active ? Rr[a][h] - (nextActive ? RTn[a][h] : Acc(0)) : Acc(0);
    }
  }
  for (int delta = 1; delta < NL; delta *= 2) {
    Acc Bi[r][r];
    spd_inverse<r, Acc>(B, Bi);
    lds_put<r, r, NL>(xs, 0, Bi, L);
    lds_put<r, r, NL>(xs, RR, A, L);
    lds_put<r, r, NL>(xs, 2 * RR, Cc, L);
    lds_put<r, CB, NL>(xs, 3 * RR, d, L);
    __syncthreads();
    Acc Bim[r][r], Am[r][r], Cm[r][r], dm[r][CB];
    Acc Bip[r][r], Ap[r][r], Cp[r][r], dp[r][CB];
    const bool up = L >= delta, dn = L + delta < NL;
    lds_get<r, r, NL>(xs, 0, Bim, L - delta, up);
    lds_get<r, r, NL>(xs, RR, Am, L - delta, up);
    lds_get<r, r, NL>(xs, 2 * RR, Cm, L - delta, up);
    lds_get<r, CB, NL>(xs, 3 * RR, dm, L - delta, up);
    lds_get<r, r, NL>(xs, 0, Bip, L + delta, dn);
    lds_get<r, r, NL>(xs, RR, Ap, L + delta, dn);
    lds_get<r, r, NL>(xs, 2 * RR, Cp, L + delta, dn);
    lds_get<r, CB, NL>(xs, 3 * RR, dp, L + delta, dn);
    __syncthreads();
    Acc al[r][r], ga[r][r];
    mm<r, r, r, Acc>(A, Bim, al);
    mm<r, r, r, Acc>(Cc, Bip, ga);
    Acc An[r][r], Cn[r][r], t1[r][r], t2[r][r], e1[r][CB], e2[r][CB];
    mm<r, r, r, Acc>(al, Am, An);
    mm<r, r, r, Acc>(ga, Cp, Cn);
    mm<r, r, r, Acc>(al, Cm, t1);
    mm<r, r, r, Acc>(ga, Ap, t2);
    mm<r, r, CB, Acc>(al, dm, e1);
    mm<r, r, CB, Acc>(ga, dp, e2);
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        A[a][c] = -An[a][c];
        Cc[a][c] = -Cn[a][c];
        B[a][c] = B[a][c] - t1[a][c] - t2[a][c];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) d[a][h] = d[a][h] - e1[a][h] - e2[a][h];
    }
  }
  {
    Acc Bc[r][r];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) Bc[a][c] = B[a][c];
    chol<r, Acc>(Bc);
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) X[a][h] = d[a][h];
    chol_solve<r, CB, Acc>(Bc, X);
  }
  lds_put<r, CB, NL>(xs, 0, X, L);
  __syncthreads();
  lds_get<r, CB, NL>(xs, 0, XT, L - 1, L >= 1);
}

// LDS values per lane of iface_pcr_levels_mw.
template <int r, int CB>
constexpr int kMwSlot = 3 * r * r + r * CB;

// k_interface_pcr: one wave per strip, lane l owns separator blocks
// [l*m, min(l*m + m, P-1)); MM is the compiled maximum of m.
// U receives the separator solutions strip-major: U[(ki*(P-1) + j)*r*CB + a*CB + h].
template <int r, int CB, int MM, typename Acc, class Reader, bool COH = false, int NL = kWave>
DEV void iface_pcr_run(const Reader& rd, Acc* __restrict__ U, int P, int m, int ki,
                       Acc* xs = nullptr) {
  const int lane = NL == kWave ? (int)(threadIdx.x % kWave) : (int)threadIdx.x;
  const int n = P - 1;
  const int s = lane * m, e = min(s + m, n);
  const bool active = s < n;

  // Local bordered elimination of blocks s .. e-2 (T = block s-1 of the
  // previous lane, B = block e-1 is this lane's unknown at the PCR level).
  Acc Ls[MM][r][r], Ub[MM][r][r], Btb[MM][r][r], Rb[MM][r][CB];
  Acc S[r][r], Bt[r][r], Rr[r][CB], TT[r][r], RT[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a) {
#pragma unroll
    for (int c = 0; c < r; ++c) { TT[a][c] = Acc(0); S[a][c] = Acc(0); Bt[a][c] = Acc(0); }
#pragma unroll
    for (int h = 0; h < CB; ++h) { RT[a][h] = Acc(0); Rr[a][h] = Acc(0); }
  }
  if (active) {
    rd.diag(s, S);
    rd.rhs(s, Rr);
    if (s > 0) {
      Acc U0[r][r];
      rd.off(s - 1, U0);
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Bt[a][c] = U0[c][a];
    }
  }
#pragma unroll
  for (int i = 0; i < MM - 1; ++i) {
    const int b = s + i;
    if (active && b < e - 1) {
      Acc Lc[r][r];
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Lc[a][c] = S[a][c];
      chol<r, Acc>(Lc);
      Acc Uc[r][r];
      rd.off(b, Uc);
      Acc V[r][r], Y[r][r], wv[r][CB];
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int c = 0; c < r; ++c) { V[a][c] = Uc[a][c]; Y[a][c] = Bt[a][c]; }
#pragma unroll
        for (int h = 0; h < CB; ++h) wv[a][h] = Rr[a][h];
      }
      chol_solve<r, r, Acc>(Lc, V);    // S^-1 U
      chol_solve<r, r, Acc>(Lc, Y);    // S^-1 Bt
      chol_solve<r, CB, Acc>(Lc, wv);  // S^-1 R
      // TT += Bt^T S^-1 Bt, RT += Bt^T S^-1 R
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int c = 0; c < r; ++c) {
          Acc v = Acc(0);
#pragma unroll
          for (int t = 0; t < r; ++t) v += Bt[t][a] * Y[t][c];
          TT[a][c] += v;
        }
#pragma unroll
        for (int h = 0; h < CB; ++h) {
          Acc v = Acc(0);
#pragma unroll
          for (int t = 0; t < r; ++t) v += Bt[t][a] * wv[t][h];
          RT[a][h] += v;
        }
      }
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int c = 0; c < r; ++c) { Ls[i][a][c] = Lc[a][c]; Ub[i][a][c] = Uc[a][c]; Btb[i][a][c] = Bt[a][c]; }
#pragma unroll
        for (int h = 0; h < CB; ++h) Rb[i][a][h] = Rr[a][h];
      }
      // next block
      Acc Sn[r][r], Rn[r][CB], Bn[r][r];
      rd.diag(b + 1, Sn);
      rd.rhs(b + 1, Rn);
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Bn[a][c] = Acc(0);
      sub_AtB<r, r, r, Acc>(Uc, V, Sn);
      sub_AtB<r, r, r, Acc>(Uc, Y, Bn);
      sub_AtB<r, r, CB, Acc>(Uc, wv, Rn);
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int c = 0; c < r; ++c) { S[a][c] = Sn[a][c]; Bt[a][c] = Bn[a][c]; }
#pragma unroll
        for (int h = 0; h < CB; ++h) Rr[a][h] = Rn[a][h];
      }
    }
  }

  Acc X[r][CB], XT[r][CB];
  if constexpr (NL == kWave)
    iface_pcr_levels<r, CB, Acc>(S, Bt, Rr, TT, RT, active, m, n, lane, X, XT);
  else
    iface_pcr_levels_mw<r, CB, Acc, NL>(S, Bt, Rr, TT, RT, active, m, n, lane, xs, X, XT);
  if (!active) return;
  Acc* out = U + (size_t)ki * n * r * CB;
#pragma unroll
  for (int a = 0; a < r; ++a)
#pragma unroll
    for (int h = 0; h < CB; ++h) st_if<COH>(out + (size_t)(e - 1) * r * CB + a * CB + h, X[a][h]);
  // back substitution: x_b = S_b^-1 (R_b - U_b x_{b+1} - Bt_b x_T)
  Acc xn[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a)
#pragma unroll
    for (int h = 0; h < CB; ++h) xn[a][h] = X[a][h];
#pragma unroll
  for (int i = MM - 2; i >= 0; --i) {
    const int b = s + i;
    if (b < e - 1) {
      Acc v[r][CB];
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int h = 0; h < CB; ++h) {
          Acc t = Rb[i][a][h];
#pragma unroll
          for (int c = 0; c < r; ++c) t -= Ub[i][a][c] * xn[c][h] + Btb[i][a][c] * XT[c][h];
          v[a][h] = t;
        }
      chol_solve<r, CB, Acc>(Ls[i], v);
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int h = 0; h < CB; ++h) {
          st_if<COH>(out + (size_t)b * r * CB + a * CB + h, v[a][h]);
          xn[a][h] = v[a][h];
        }
    }
  }
}

// The solver of one strip: its chunk records prefetched into registers
// when the lane's run fits (MM + 1 records), else read as needed.
template <int r, int CB, int MM, typename Acc, bool COH = false>
DEV void iface_pcr_strip(const Acc* __restrict__ sum, Acc* __restrict__ U, int P, int m, int ki) {
  using LY = IfaceLayout<r, CB>;
  const Acc* S = sum + (size_t)ki * P * LY::F;
  if constexpr ((MM + 1) * LY::F <= 160) {
    PreReader<r, CB, MM + 1, Acc, COH> rd;
    rd.load(S, (int)(threadIdx.x % kWave) * m, P, m + 1);
    iface_pcr_run<r, CB, MM, Acc, PreReader<r, CB, MM + 1, Acc, COH>, COH>(rd, U, P, m, ki);
  } else {
    const SepReader<r, CB, Acc, COH> rd{S, P};
    iface_pcr_run<r, CB, MM, Acc, SepReader<r, CB, Acc, COH>, COH>(rd, U, P, m, ki);
  }
}

template <int r, int CB, int MM, typename Acc>
__global__ __launch_bounds__(kWave) void k_interface_pcr(const Acc* __restrict__ sum,
                                                         Acc* __restrict__ U, int nK, int P,
                                                         int m, long long zi, long long zu) {
  const int z = blockIdx.z;   // image of a batched launch (summaries zi, solutions zu bytes apart)
  iface_pcr_strip<r, CB, MM, Acc>(zmove_bytes(sum, zi, z), zmove_bytes(U, zu, z), P, m, blockIdx.x);
}

// Register solver on a workgroup of NL lanes per strip (cyclic reduction
// through LDS): for runs too long for one wave's registers (r = 3), where NL
// lanes cut every lane's run to at most MM blocks, so that no scratch round
// trip is needed.  Records are read as needed (no prefetch: registers).
constexpr int kMwMM = 4;
template <int r, int CB, typename Acc, int NL>
__global__ __launch_bounds__(NL) void k_interface_pcr_mw(const Acc* __restrict__ sum,
                                                         Acc* __restrict__ U, int P, int m,
                                                         long long zi, long long zu) {
  using LY = IfaceLayout<r, CB>;
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  const SepReader<r, CB, Acc> rd{zmove_bytes(sum, zi, z) + (size_t)blockIdx.x * P * LY::F, P};
  iface_pcr_run<r, CB, kMwMM, Acc, SepReader<r, CB, Acc>, false, NL>(
      rd, zmove_bytes(U, zu, z), P, m, blockIdx.x, reinterpret_cast<Acc*>(smem));
}

// Scratch values per separator block kept by iface_pcr_strip_long: the
// Cholesky factor of the pivot block, the coupling to the next block, the
// coupling to the previous lane's block and the right-hand side.
template <int r, int CB>
constexpr int kLongSlot = 3 * r * r + r * CB;

// iface_pcr_strip for runs of any length: the same elimination, cyclic
// reduction and back substitution, with the per-block values of each lane's
// run kept in global scratch instead of registers (layout: strip ki, block i
// of the run, value f, lane -> scr[((ki * m + i) * kLongSlot + f) * NL + lane],
// so that a wave's accesses are contiguous).  Used when the runs are longer
// than the register version holds (long lines at r >= 3).  NL lanes solve one
// strip: one wave (NL = 64, cyclic reduction by lane shuffles) or a workgroup
// of NL / 64 waves (cyclic reduction through LDS at xs), which shortens every
// lane's run where the strips alone leave the GPU underfilled.
template <int r, int CB, typename Acc, int NL = kWave>
DEV void iface_pcr_strip_long(const Acc* __restrict__ sum, Acc* __restrict__ U, int P, int m,
                              int ki, Acc* __restrict__ scr, Acc* xs = nullptr) {
  using LY = IfaceLayout<r, CB>;
  constexpr int FS = kLongSlot<r, CB>;
  const int lane = NL == kWave ? (int)(threadIdx.x % kWave) : (int)threadIdx.x;
  const int n = P - 1;
  const int s = lane * m, e = min(s + m, n);
  const bool active = s < n;
  SepReader<r, CB, Acc> rd{sum + (size_t)ki * P * LY::F, P};
  Acc* slots = scr + (size_t)ki * m * FS * NL + lane;
  auto at = [&](int i, int f) -> Acc& { return slots[((size_t)i * FS + f) * NL]; };

  Acc S[r][r], Bt[r][r], Rr[r][CB], TT[r][r], RT[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a) {
#pragma unroll
    for (int c = 0; c < r; ++c) { TT[a][c] = Acc(0); S[a][c] = Acc(0); Bt[a][c] = Acc(0); }
#pragma unroll
    for (int h = 0; h < CB; ++h) { RT[a][h] = Acc(0); Rr[a][h] = Acc(0); }
  }
  if (active) {
    rd.diag(s, S);
    rd.rhs(s, Rr);
    if (s > 0) {
      Acc U0[r][r];
      rd.off(s - 1, U0);
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Bt[a][c] = U0[c][a];
    }
  }
  const int run = active ? e - 1 - s : 0;   // blocks eliminated locally
  // The coupling of block b and the diagonal and right-hand side of block b+1
  // are loaded one iteration ahead, so their latency overlaps the current
  // block's elimination.
  Acc Uc[r][r], Sn[r][r], Rn[r][CB];
  if (run > 0) {
    rd.off(s, Uc);
    rd.diag(s + 1, Sn);
    rd.rhs(s + 1, Rn);
  }
  for (int i = 0; i < run; ++i) {
    Acc Uc2[r][r], Sn2[r][r], Rn2[r][CB];
    if (i + 1 < run) {
      rd.off(s + i + 1, Uc2);
      rd.diag(s + i + 2, Sn2);
      rd.rhs(s + i + 2, Rn2);
    }
    Acc Lc[r][r];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) Lc[a][c] = S[a][c];
    chol<r, Acc>(Lc);
    Acc V[r][r], Y[r][r], wv[r][CB];
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) { V[a][c] = Uc[a][c]; Y[a][c] = Bt[a][c]; }
#pragma unroll
      for (int h = 0; h < CB; ++h) wv[a][h] = Rr[a][h];
    }
    chol_solve<r, r, Acc>(Lc, V);    // S^-1 U
    chol_solve<r, r, Acc>(Lc, Y);    // S^-1 Bt
    chol_solve<r, CB, Acc>(Lc, wv);  // S^-1 R
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        Acc v = Acc(0);
#pragma unroll
        for (int t = 0; t < r; ++t) v += Bt[t][a] * Y[t][c];
        TT[a][c] += v;
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        Acc v = Acc(0);
#pragma unroll
        for (int t = 0; t < r; ++t) v += Bt[t][a] * wv[t][h];
        RT[a][h] += v;
      }
    }
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        at(i, a * r + c) = Lc[a][c];
        at(i, r * r + a * r + c) = Uc[a][c];
        at(i, 2 * r * r + a * r + c) = Bt[a][c];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) at(i, 3 * r * r + a * CB + h) = Rr[a][h];
    }
    Acc Bn[r][r];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) Bn[a][c] = Acc(0);
    sub_AtB<r, r, r, Acc>(Uc, V, Sn);
    sub_AtB<r, r, r, Acc>(Uc, Y, Bn);
    sub_AtB<r, r, CB, Acc>(Uc, wv, Rn);
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        S[a][c] = Sn[a][c];
        Bt[a][c] = Bn[a][c];
        Uc[a][c] = Uc2[a][c];
        Sn[a][c] = Sn2[a][c];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        Rr[a][h] = Rn[a][h];
        Rn[a][h] = Rn2[a][h];
      }
    }
  }

  Acc X[r][CB], XT[r][CB];
  if constexpr (NL == kWave)
    iface_pcr_levels<r, CB, Acc>(S, Bt, Rr, TT, RT, active, m, n, lane, X, XT);
  else
    iface_pcr_levels_mw<r, CB, Acc, NL>(S, Bt, Rr, TT, RT, active, m, n, lane, xs, X, XT);
  if (!active) return;
  Acc* out = U + (size_t)ki * n * r * CB;
#pragma unroll
  for (int a = 0; a < r; ++a)
#pragma unroll
    for (int h = 0; h < CB; ++h) out[(size_t)(e - 1) * r * CB + a * CB + h] = X[a][h];
  Acc xn[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a)
#pragma unroll
    for (int h = 0; h < CB; ++h) xn[a][h] = X[a][h];
  // back substitution x_b = S_b^-1 (R_b - U_b x_{b+1} - Bt_b x_T), the
  // scratch values of block i-1 loaded while block i is solved
  Acc cur[FS];
  if (run > 0) {
#pragma unroll
    for (int f = 0; f < FS; ++f) cur[f] = at(run - 1, f);
  }
  for (int i = run - 1; i >= 0; --i) {
    Acc nxt[FS];
    if (i > 0) {
#pragma unroll
      for (int f = 0; f < FS; ++f) nxt[f] = at(i - 1, f);
    }
    Acc Lc[r][r], v[r][CB];
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) Lc[a][c] = cur[a * r + c];
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        Acc t = cur[3 * r * r + a * CB + h];
#pragma unroll
        for (int c = 0; c < r; ++c)
          t -= cur[r * r + a * r + c] * xn[c][h] + cur[2 * r * r + a * r + c] * XT[c][h];
        v[a][h] = t;
      }
    }
    chol_solve<r, CB, Acc>(Lc, v);
    const int b = s + i;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        out[(size_t)b * r * CB + a * CB + h] = v[a][h];
        xn[a][h] = v[a][h];
      }
#pragma unroll
    for (int f = 0; f < FS; ++f) cur[f] = nxt[f];
  }
}

template <int r, int CB, typename Acc, int NL>
__global__ __launch_bounds__(NL) void k_interface_pcr_long(const Acc* __restrict__ sum,
                                                           Acc* __restrict__ U,
                                                           Acc* __restrict__ scr, int P, int m,
                                                           long long zi, long long zu) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  iface_pcr_strip_long<r, CB, Acc, NL>(zmove_bytes(sum, zi, z), zmove_bytes(U, zu, z), P, m,
                                       blockIdx.x, zmove_bytes(scr, zi, z),
                                       reinterpret_cast<Acc*>(smem));
}

// ---------------------------------------------------------------------------
// k_expand: final solve of every chunk with its separators known, scatter and
// average.  Block (x, y) owns pass columns [x*OW, x*OW + OW) and rows of chunks
// [y*Q, y*Q + Q); its 64 lanes are the strips whose columns touch them.
//
// Backward (MODE = kModeBackward): the chunk is solved for the pass solution u
// (right-hand sides X) and the adjoint solution ubar (right-hand sides X2 /
// cover count) together.  Y receives the scattered sum of ubar (the input
// gradient; the averaging was already applied to X2).  Every edge (p, q) of
// the subsystem with q in the chunk (p may be one of the previous chunk's
// last r elements, known from the separator solve) contributes
// t = -sum_c (ubar_p - ubar_q)(u_p - u_q): omega t to the lambda gradient and
// lambda t d omega / d(G_p - G_q) (+ at p, - at q) to the guidance gradient.
// Terms of the previous chunk's elements go to bw.side (added by the fix-up
// kernel); lambda partials go to bw.lpart, one per block, from the strips
// the block owns (a strip is solved by the two blocks whose columns it
// touches, and owned by the first).
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE,
          bool DIRECT = false, bool COH = false, bool KEEP = false, bool GT = false>
DEV void expand_tile(const float* __restrict__ G, float* __restrict__ Y, const PassGeom& geo,
                     const WeightParams& wp, float lam_in, int c0, const Acc* __restrict__ Us,
                     int OW, int pch, const BwdArgs& bw, int bx, int by, int nbx, float* smem,
                     const PlaneSrc<CB>* src = nullptr);

template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE>
DEV void expand_block(const float* __restrict__ X, const float* __restrict__ G,
                      float* __restrict__ Y, const PassGeom& geo, const WeightParams& wp,
                      float lam_in, int c0, const Acc* __restrict__ Us, int OW, int pitch,
                      const BwdArgs& bw, int bx, int by, int nbx, float* smem) {
  constexpr bool BWD = MODE == kModeBackward;
  constexpr int NR = BWD ? 2 * CB : CB;   // right-hand sides
  using CV = ChunkView<r, R, S1>;
  constexpr int TA = Q * R + 2;
  const int lane = threadIdx.x % kWave;
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int ki_lo = expand_first_strip(bx, OW, geo, r);
  const int colbase = centre_of(ki_lo, geo, r) - r;
  const int a_lo = by * Q * R;
  const int TB = S1 ? kWave + 2 * r : tile_width<r>(geo.stride);
  const int pch = S1 ? CV::PITCH1 : pitch;
  const PlaneSrc<CB> src{X, bw.ybar, c0, (int)geo.plane};
  if constexpr (S1)
    load_tile_s1<r, NR, CB, TA, Q>(smem, G, src, geo, a_lo, colbase, pch, lane, wq);
  else
    load_tile<NR, CB, TA, kWave * Q, 8>(smem, G, src, geo, a_lo, colbase, TB, pch, threadIdx.x);
  __syncthreads();
  expand_tile<r, CB, R, Q, S1, KIND, Acc, MODE>(G, Y, geo, wp, lam_in, c0, Us, OW, pch, bw, bx,
                                                by, nbx, smem);
}

// Transposed store of a block's staged rows: LDS row tr (pitch kWave + 1,
// one bank of padding), column bb - colbase, holds output (a_lo + tr, bb),
// which goes to Yc[h*plane + bb*L + a_lo + tr].  A column's rows are
// contiguous in the output, so consecutive threads take consecutive rows of
// one column (the block's Q waves share the work): four rows per 16-byte
// store when the runs are 16-byte aligned (a_lo is a multiple of QR), one row
// per store otherwise.  GTP: staged plane CB holds the guidance, which goes to
// gT[bb*L + a_lo + tr].
template <int CB, int Q, int R, bool GTP = false>
DEV void store_transposed(const float* smem, float* __restrict__ Yc, const float* Ybase, int plane,
                          int L, int a_lo, int arows, int b_lo, int b_hi, int colbase,
                          float* __restrict__ gT = nullptr) {
  constexpr int RP = kWave + 1, QR = Q * R, nthr = kWave * Q;
  const int ncols = b_hi - b_lo;
  if (QR % 4 == 0 && L % 4 == 0 && arows % 4 == 0 && plane % 4 == 0 &&
      (reinterpret_cast<uintptr_t>(Ybase) & 15) == 0 &&
      (!GTP || (reinterpret_cast<uintptr_t>(gT) & 15) == 0)) {
    const int q4 = arows / 4;
    for (int idx = threadIdx.x; idx < q4 * ncols; idx += nthr) {
      const int bc = idx / q4, tr = 4 * (idx - bc * q4);
      const int bb = b_lo + bc;
      const float* cell = smem + tr * RP + (bb - colbase);
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        const float* c = cell + h * QR * RP;
        *reinterpret_cast<float4*>(Yc + h * plane + (size_t)bb * L + a_lo + tr) =
            make_float4(c[0], c[RP], c[2 * RP], c[3 * RP]);
      }
      if constexpr (GTP) {
        const float* c = cell + CB * QR * RP;
        *reinterpret_cast<float4*>(gT + (size_t)bb * L + a_lo + tr) =
            make_float4(c[0], c[RP], c[2 * RP], c[3 * RP]);
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < arows * ncols; idx += nthr) {
      const int bc = idx / arows, tr = idx - bc * arows;
      const int bb = b_lo + bc;
      const float* cell = smem + tr * RP + (bb - colbase);
#pragma unroll
      for (int h = 0; h < CB; ++h) Yc[h * plane + (size_t)bb * L + a_lo + tr] = cell[h * QR * RP];
      if constexpr (GTP) gT[(size_t)bb * L + a_lo + tr] = cell[CB * QR * RP];
    }
  }
}

// The solve and output of a block whose tile is in LDS (see expand_block), or,
// with DIRECT, whose chunks are read from global memory (stride-1 column pass).
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE, bool DIRECT,
          bool COH, bool KEEP, bool GT>
DEV void expand_tile(const float* __restrict__ G, float* __restrict__ Y, const PassGeom& geo,
                     const WeightParams& wp, float lam_in, int c0, const Acc* __restrict__ Us,
                     int OW, int pch, const BwdArgs& bw, int bx, int by, int nbx, float* smem,
                     const PlaneSrc<CB>* src) {
  constexpr bool BWD = MODE == kModeBackward;
  constexpr int NR = BWD ? 2 * CB : CB;   // right-hand sides
  constexpr int NO = BWD ? CB + 1 : CB;   // output planes (backward: + guidance gradient)
  using CV = ChunkView<r, R, S1>;
  constexpr int E = CV::E, w = CV::w;
  constexpr int TA = Q * R + 2;
  const int lane = threadIdx.x % kWave;
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int b_lo = bx * OW, b_hi = min(b_lo + OW, geo.W);
  const int ki_lo = expand_first_strip(bx, OW, geo, r);
  const int colbase = centre_of(ki_lo, geo, r) - r;
  const int j0 = by * Q, j = j0 + wq;
  const int a_lo = j0 * R;
  const int TB = S1 ? kWave + 2 * r : tile_width<r>(geo.stride);
  const int ki = ki_lo + lane;
  const bool active = ki < geo.nK && j < geo.P;
  const bool hasT = j > 0, hasB = j + 1 < geo.P;
  const int k = active ? centre_of(ki, geo, r) : colbase + r;
  const int rows = max(0, min(R, geo.L - j * R));
  const bool want_edges = BWD && (bw.gbar != nullptr || bw.lpart != nullptr);

  Acc Z[E][NR];     // z = D^{-1} L^{-1} f, overwritten by the solution u
  Acc Lf[E][r];     // Lf[m][a-1] = L(m+a, m)
  Acc uT[r][NR], uB[r][NR];
  float gv[E + 2 * r];
  float om[E + r][r];
  const float lam = lam_in;
  // Forward direct stride-1 column pass: each output row is stored as soon as
  // its back substitution is done, so the stores drain during the rest of it.
  constexpr bool ROWWISE = DIRECT && !BWD && S1;
  if (active) {
    // Separator values first: their loads are the head of the dependency chain.
    const int n_sep = geo.P - 1;
    bool split = false;
    if constexpr (BWD) {
      if (bw.useps) {
        // the pass solution's separators saved by the forward, the adjoint's
        // from this pass's own interface (r x CB each)
        split = true;
        const Acc* uf = reinterpret_cast<const Acc*>(bw.useps) + (size_t)ki * n_sep * r * CB;
        const Acc* ua = Us + (size_t)ki * n_sep * r * CB;
#pragma unroll
        for (int a = 0; a < r; ++a)
#pragma unroll
          for (int h = 0; h < CB; ++h) {
            const size_t oT = (size_t)(j - 1) * r * CB + a * CB + h;
            const size_t oB = (size_t)j * r * CB + a * CB + h;
            uT[a][h] = hasT ? uf[oT] : Acc(0);
            uB[a][h] = hasB ? uf[oB] : Acc(0);
            uT[a][CB + h] = hasT ? ua[oT] : Acc(0);
            uB[a][CB + h] = hasB ? ua[oB] : Acc(0);
          }
      }
    }
    if (!split) {
      const Acc* us = Us + (size_t)ki * n_sep * r * NR;
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          uT[a][h] = hasT ? ld_if<COH>(us + (size_t)(j - 1) * r * NR + a * NR + h) : Acc(0);
          uB[a][h] = hasB ? ld_if<COH>(us + (size_t)j * r * NR + a * NR + h) : Acc(0);
        }
    }
    typename std::conditional<DIRECT, GlobalChunk<r, R, NR>, CV>::type cv;
    if constexpr (DIRECT) {
      cv.init(G, *src, geo, j * R, k);
    } else {
      cv.base = smem + (wq * R + 1) * pch + (k - colbase);
      cv.pitch = pch;
      cv.plane = TA * pch;
      cv.a0 = j * R;
      cv.L = geo.L;
    }
    float fpre[DIRECT ? E : 1][NR];   // see reduce_tile
    if constexpr (DIRECT) {
#pragma unroll
      for (int m = 0; m < E; ++m)
#pragma unroll
        for (int c = 0; c < NR; ++c) fpre[m][c] = cv.f(m, c);
    }
    float lw[E + r][r];
    if constexpr (BWD) {
      chunk_omega<r, KIND>(cv, wp, gv, om);
#pragma unroll
      for (int m = 0; m < E + r; ++m)
#pragma unroll
        for (int d = 0; d < r; ++d) lw[m][d] = lam * om[m][d];
    } else {
      float lamS[r + 1];
#pragma unroll
      for (int d = 0; d <= r; ++d) lamS[d] = lam * wp.spatial[d];
      chunk_weights<r, KIND>(cv, wp, lamS, lw);
    }
    float ic[2 * r + 1];
    if constexpr (BWD) inv_counts<r, S1>(k, geo, ic);
    auto fval = [&](int m, int c) -> Acc {   // 0 outside the subsystem
      const float v = DIRECT ? fpre[DIRECT ? m : 0][c] : cv.f(m, c);
      if (BWD && c >= CB) return Acc(v * ic[col_of<r>(m) + r]);
      return Acc(v);
    };
    Acc W[r + 1][r + 1];
    Acc Rw[r + 1][NR];
#pragma unroll
    for (int a = 0; a < r; ++a) {
      W[a][a] = diag_at<r, E, Acc>(lw, a);
#pragma unroll
      for (int b = 0; b < a; ++b) W[a][b] = -Acc(lw[b + r][a - b - 1]);
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        Acc v = fval(a, h);
#pragma unroll
        for (int c = a; c < r; ++c) v += Acc(lw[c][a + r - c - 1]) * uT[c][h];
        Rw[a][h] = v;
      }
    }
    auto step = [&](const int m) {
      const int n = m + r;
      bool dummy = true;
      if (hasB && n >= E - r) {
        // n belongs to the known separator S_j: its coupling moves to the RHS.
        const int bi = n - (E - r);
#pragma unroll
        for (int b = 0; b < r; ++b)
#pragma unroll
          for (int h = 0; h < NR; ++h) Rw[b][h] += Acc(lw[m + b + r][r - b - 1]) * uB[bi][h];
      } else if (n < E) {
        dummy = false;
        W[r][r] = diag_at<r, E, Acc>(lw, n);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = -Acc(lw[m + b + r][r - b - 1]);
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[r][h] = fval(n, h);
      }
      if (dummy) {
        W[r][r] = Acc(1);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = Acc(0);
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[r][h] = Acc(0);
      }
      const Acc invD = recip(W[0][0]);
      Acc l[r + 1];
#pragma unroll
      for (int a = 1; a <= r; ++a) {
        l[a] = W[a][0] * invD;
        Lf[m][a - 1] = l[a];
      }
#pragma unroll
      for (int h = 0; h < NR; ++h) Z[m][h] = Rw[0][h] * invD;
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int b = 1; b <= a; ++b) W[a][b] -= l[a] * W[b][0];
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[a][h] -= l[a] * Rw[0][h];
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) W[a][b] = W[a + 1][b + 1];
#pragma unroll
        for (int h = 0; h < NR; ++h) Rw[a][h] = Rw[a + 1][h];
      }
    };
#pragma unroll
    for (int m = 0; m < E - r; ++m) step(m);
    if (!hasB) {
#pragma unroll
      for (int m = E - r; m < E; ++m) step(m);
    } else {
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int h = 0; h < NR; ++h) Z[E - r + a][h] = uB[a][h];
#pragma unroll
        for (int t = 0; t < r; ++t) Lf[E - r + a][t] = Acc(0);
      }
    }
    // back substitution u_m = z_m - sum_a L(m+a, m) u_{m+a}
#pragma unroll
    for (int m = E - 1; m >= 0; --m) {
      if (!ROWWISE && (m < E - r || !hasB)) {
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          Acc v = Z[m][h];
#pragma unroll
          for (int a = 1; a <= r; ++a)
            if (m + a < E) v -= Lf[m][a - 1] * Z[m + a][h];
          Z[m][h] = v;
        }
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
      for (int h = 0; h < NR; ++h) Z[m][h] = Acc(0);
  }

  // Backward edge terms (guidance gradient per element, lambda partial).
  float Gv[BWD ? E + r : 1];
  double lsum = 0.0;
  if constexpr (BWD) {
#pragma unroll
    for (int m = 0; m < E + r; ++m) Gv[m] = 0.0f;
    const int ki_next = bx + 1 < nbx ? expand_first_strip(bx + 1, OW, geo, r) : geo.nK;
    const bool owns = ki < ki_next;
    if (active && want_edges) {
#pragma unroll
      for (int q = 0; q < E; ++q)
#pragma unroll
        for (int d = 1; d <= r; ++d) {
          const int p = q - d;
          if (p >= -r) {
            Acc t = Acc(0);
#pragma unroll
            for (int h = 0; h < CB; ++h) {
              const Acc up = p < 0 ? uT[p + r][h] : Z[p][h];
              const Acc bp = p < 0 ? uT[p + r][CB + h] : Z[p][CB + h];
              t -= (bp - Z[q][CB + h]) * (up - Z[q][h]);
            }
            const float wpq = om[p + r][d - 1];
            if (owns) lsum += double(wpq) * double(t);
            const float kap = float(Acc(lam) * t) * domega<KIND>(wpq, gv[p + r] - gv[q + r], wp);
            Gv[p + r] += kap;
            Gv[q + r] -= kap;
          }
        }
    }
    if (bw.lpart) {
      __shared__ double lred[16];
      double v = lsum;
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
      if (lane == 0) lred[wq] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += lred[i];
        bw.lpart[(size_t)by * nbx + bx] = s;
      }
    }
  }
  const bool wantg = BWD && bw.gbar != nullptr;
  // value of output plane o at element m of this lane's strip
  auto outval = [&](int m, int o) -> float {
    if constexpr (BWD) return o < CB ? float(Z[m][CB + o]) : Gv[m + r];
    return float(Z[m][o]);
  };

  const int nrow = Q * R;
  const int arows = max(0, min(nrow, geo.L - a_lo));
  const int plane = (int)geo.plane;
  float* Yc = Y + c0 * plane;
  if constexpr (S1) {
    // Lane l outputs column b = colbase + l.  The strips covering it are the
    // lanes l-2r..l (centres b+r..b-r); lane l-t holds column b at row-vector
    // position t on even rows and 2r-t on odd rows.  Lanes without a strip
    // contribute 0 (including those left of lane 0).  The sum is a fixed
    // nesting of one-lane wave shifts, so it is reproducible.
    const int b = colbase + lane;
    const bool own = b >= b_lo && b < b_hi && j < geo.P;
    float inv = 1.0f;
    if constexpr (!BWD) {
      const int cnt = min(geo.W - 1 - r, b + r) - max(r, b - r) + 1;
      inv = __builtin_amdgcn_rcpf(float(max(cnt, 1)));
    }
    if constexpr (ROWWISE) {
      // KEEP: separators of another cut (seps_R rows per chunk) kept for the
      // backward: the last r elements of every subsystem row that ends one of
      // its chunks, stored by the block that owns the strip.
      bool keep_seps = false;
      if constexpr (KEEP) {
        const int ki_next = bx + 1 < nbx ? expand_first_strip(bx + 1, OW, geo, r) : geo.nK;
        keep_seps = bw.seps_out != nullptr && active && ki < ki_next;
      }
#pragma unroll
      for (int rho = R - 1; rho >= 0; --rho) {
        if (active) {
#pragma unroll
          for (int m = rho * w + w - 1; m >= rho * w; --m) {
            if (m < E - r || !hasB) {
#pragma unroll
              for (int h = 0; h < NR; ++h) {
                Acc v = Z[m][h];
#pragma unroll
                for (int a = 1; a <= r; ++a)
                  if (m + a < E) v -= Lf[m][a - 1] * Z[m + a][h];
                Z[m][h] = v;
              }
            }
          }
        }
        if (KEEP && keep_seps) {
          const int rows_to = j * R + rho + 1;   // subsystem rows up to this one
          const int js = rows_to / bw.seps_R - 1;
          if (rows_to % bw.seps_R == 0 && js < bw.seps_n) {
            Acc* o = reinterpret_cast<Acc*>(bw.seps_out) + ((size_t)ki * bw.seps_n + js) * r * CB;
#pragma unroll
            for (int a = 0; a < r; ++a)
#pragma unroll
              for (int h = 0; h < CB; ++h) o[a * CB + h] = Z[rho * w + w - r + a][h];
          }
        }
        float orow[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          float acc = outval(rho * w + ((rho & 1) ? 0 : 2 * r), o);
#pragma unroll
          for (int t = 2 * r - 1; t >= 0; --t)
            acc = outval(rho * w + ((rho & 1) ? 2 * r - t : t), o) + lane_shr1(acc);
          orow[o] = acc * inv;
        }
        if (geo.out_t) {           // stage the row for the transposed store below
#pragma unroll
          for (int h = 0; h < CB; ++h) smem[(h * Q * R + wq * R + rho) * (kWave + 1) + lane] = orow[h];
          if constexpr (GT) {      // and the guidance at the lane's output column
            const int row = j * R + rho;
            smem[(CB * Q * R + wq * R + rho) * (kWave + 1) + lane] =
                (row < geo.L && b < geo.W) ? G[(size_t)row * geo.sa + b] : 0.0f;
          }
        } else if (own && rho < rows) {
          const int o = (j * R + rho) * (int)geo.sa + b;
#pragma unroll
          for (int h = 0; h < CB; ++h) Yc[h * plane + o] = orow[h];
        }
      }
      if (geo.out_t) {
        __syncthreads();
        store_transposed<CB, Q, R, GT>(smem, Yc, Y, plane, geo.L, a_lo, arows, b_lo, b_hi,
                                       colbase, bw.gT_out);
      }
      return;
    }
    float out[R][NO];
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        // sum_t shift_t(v_t) evaluated as v_0 + shift(v_1 + shift(v_2 + ...))
        float acc = outval(rho * w + ((rho & 1) ? 0 : 2 * r), o);
#pragma unroll
        for (int t = 2 * r - 1; t >= 0; --t)
          acc = outval(rho * w + ((rho & 1) ? 2 * r - t : t), o) + lane_shr1(acc);
        out[rho][o] = acc * inv;
      }
    if constexpr (BWD) {
      // The previous chunk's last row is odd: its element -r+i (i < r) lies in
      // column k-1-i, so column b gathers element -r+i of lane l-r+1+i.
      if (wantg) {
        float sacc = Gv[0];
#pragma unroll
        for (int i = 1; i < r; ++i) sacc = Gv[i] + lane_shr1(sacc);
        if (own && hasT) {
          float* sp = bw.side + (size_t)j * geo.W + b;
          *sp = bw.sacc ? *sp + sacc : sacc;
        }
      }
    }
    if (geo.sb == 1) {   // column pass: lanes write consecutive columns of each row
      if (own) {
#pragma unroll
        for (int rho = 0; rho < R; ++rho)
          if (rho < rows) {
            const int o = (j * R + rho) * (int)geo.sa + b;
            if (geo.out_t) {   // staged for the transposed store below
#pragma unroll
              for (int h = 0; h < CB; ++h)
                smem[(h * Q * R + wq * R + rho) * (kWave + 1) + lane] = out[rho][h];
            } else {
#pragma unroll
              for (int h = 0; h < CB; ++h) Yc[h * plane + o] = out[rho][h];
            }
            if constexpr (BWD) {   // the guidance gradient stays in the frame of the pass
              if (wantg) bw.gbar[o] = (bw.gacc ? bw.gbar[o] : 0.0f) + out[rho][CB];
            }
          }
      }
      if (geo.out_t) {
        __syncthreads();
        store_transposed<CB, Q, R>(smem, Yc, Y, plane, geo.L, a_lo, arows, b_lo, b_hi, colbase);
      }
    } else {             // row pass: transpose through the (consumed) image planes
      if (own) {
#pragma unroll
        for (int rho = 0; rho < R; ++rho)
#pragma unroll
          for (int o = 0; o < NO; ++o)
            smem[(o + 1) * TA * pch + (wq * R + 1 + rho) * pch + lane] = out[rho][o];
      }
      __syncthreads();
      const int ncols = b_hi - b_lo;
      for (int idx = threadIdx.x; idx < arows * ncols; idx += kWave * Q) {
        const int bc = idx / arows, tr = idx - bc * arows;
        const int bb = b_lo + bc, a = a_lo + tr;
        const float* cell = smem + TA * pch + (tr + 1) * pch + (bb - colbase);
        const int o = a + bb * (int)geo.sb;
#pragma unroll
        for (int h = 0; h < CB; ++h) Yc[h * plane + o] = cell[h * TA * pch];
        if constexpr (BWD) {
          if (wantg) bw.gbar[o] = (bw.gacc ? bw.gbar[o] : 0.0f) + cell[CB * TA * pch];
        }
      }
    }
  } else {
    // Accumulator planes: after the input tile in LDS mode (whose planes are
    // consumed), from the start of the LDS with direct reads.
    const int acc0 = DIRECT ? 0 : TA * pch;
    __syncthreads();   // all tile reads done: the image planes become accumulators
    constexpr int r0 = BWD ? 0 : 1;   // backward also accumulates the row above
    for (int p = 0; p < NO; ++p)
      for (int idx = threadIdx.x; idx < (nrow + 1 - r0) * TB; idx += kWave * Q) {
        const int ta = r0 + idx / TB, tb = idx - (ta - r0) * TB;
        smem[acc0 + p * TA * pch + ta * pch + tb] = 0.0f;
      }
    // Forward: row 0 of accumulator plane 0 (never accumulated) holds the
    // reciprocal cover count of each owned column, computed once per column.
    const int ncols = b_hi - b_lo;
    float* invc = smem + acc0;
    if constexpr (!BWD)
      for (int bc = threadIdx.x; bc < ncols; bc += kWave * Q)
        invc[bc] = 1.0f / float(cover_count(b_lo + bc, geo, r));
    __syncthreads();
    // Sum over the strips covering each pixel, in a fixed order (q = 0..2r).
#pragma unroll
    for (int q = 0; q < w; ++q) {
      if (active) {
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
          if (rho < rows) {
            const int col = ((rho & 1) ? (k + r - q) : (k - r + q)) - colbase;
            float* cell = smem + acc0 + (wq * R + 1 + rho) * pch + col;
#pragma unroll
            for (int o = 0; o < NO; ++o) cell[o * TA * pch] += outval(rho * w + q, o);
          }
        }
      }
      __syncthreads();
    }
    if constexpr (BWD) {
      // terms of the previous chunk's last row (odd: element -r+i at k-1-i)
#pragma unroll
      for (int i = 0; i < r; ++i) {
        if (active && wantg)
          smem[acc0 + (NO - 1) * TA * pch + (wq * R) * pch + (k - 1 - i - colbase)] += Gv[i];
        __syncthreads();
      }
    }
    // Row-major output walks rows; column-major output (row pass, or a
    // transposed store, pixel (a, b) at b * L + a) walks columns.  Element
    // idx = outer * n_in + inner of the walk, for idx = thread, thread + step,
    // ...: the indices advance by a fixed quotient and remainder.
    const bool colmajor = !(geo.sb == 1 && !geo.out_t);
    const int n_in = colmajor ? arows : ncols, n_out = colmajor ? ncols : arows;
    const int step = kWave * Q, dq = step / n_in, dr = step - dq * n_in;
    int outer = threadIdx.x / n_in, inner = threadIdx.x - outer * n_in;
    for (; outer < n_out; outer += dq) {
      const int tr = colmajor ? inner : outer, bc = colmajor ? outer : inner;
      inner += dr;
      if (inner >= n_in) {
        inner -= n_in;
        ++outer;
      }
      const int bb = b_lo + bc, a = a_lo + tr;
      const float inv = BWD ? 1.0f : invc[bc];
      const float* cell = smem + acc0 + (tr + 1) * pch + (bb - colbase);
      const int o = geo.out_t     ? a + bb * geo.L
                    : geo.sb == 1 ? a * (int)geo.sa + bb
                                  : a + bb * (int)geo.sb;
#pragma unroll
      for (int h = 0; h < CB; ++h) Yc[h * plane + o] = cell[h * TA * pch] * inv;
      if constexpr (BWD) {
        if (wantg) bw.gbar[o] = (bw.gacc ? bw.gbar[o] : 0.0f) + cell[CB * TA * pch];
      }
    }
    if constexpr (BWD) {
      if (wantg && j0 > 0 && j0 < geo.P)
        for (int bc = threadIdx.x; bc < ncols; bc += kWave * Q) {
          float* sp = bw.side + (size_t)j0 * geo.W + b_lo + bc;
          const float v = smem[acc0 + (NO - 1) * TA * pch + (b_lo + bc - colbase)];
          *sp = bw.sacc ? *sp + v : v;
        }
    }
  }
}

// Logical block (bx, by) of this workgroup such that each XCD runs one
// contiguous range of the row-major block order.  The dispatcher deals
// workgroups to the 8 XCDs round-robin by linear id; neighbouring blocks
// overlap in their halo columns and rows, and the overlap is an L2 hit only
// when both run on one XCD (each XCD has its own L2).
constexpr int kXcds = 8;
// Position of dispatch slot lin (of n) in that order: a bijection of [0, n).
DEV int xcd_rank(int lin, int n) {
  const int x = lin % kXcds, idx = lin / kXcds;
  const int q = n / kXcds, rem = n % kXcds;
  return x * q + min(x, rem) + idx;
}
DEV void xcd_block(int& bx, int& by) {
  const int nx = gridDim.x;
  const int logical = xcd_rank(blockIdx.y * nx + blockIdx.x, nx * gridDim.y);
  by = logical / nx;
  bx = logical - by * nx;
}

// Column-pass kernels without an LDS tile (GlobalChunk views).
template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE>
__global__ __launch_bounds__(kWave* Q) void k_reduce_d(
    const float* __restrict__ X, const float* __restrict__ X2, const float* __restrict__ G,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    Acc* __restrict__ sum) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  const PlaneSrc<CB> src{zmove(X, geo.zx, z), zmove(X2, geo.zx2, z), c0, (int)geo.plane};
  int bx, by;
  xcd_block(bx, by);
  reduce_tile<r, CB, R, Q, S1, KIND, Acc, MODE, true>(
      geo, wp, load_lambda(lam_dev, lam_host), 0, zmove_bytes(sum, geo.zi, z), bx, by, smem,
      zmove(G, geo.zg, z), &src);
}

// The backward operands of image z of a batched launch.
DEV BwdArgs bwd_at(BwdArgs bw, const PassGeom& geo, int z) {
  bw.ybar = zmove(bw.ybar, geo.zx2, z);
  bw.gbar = zmove(bw.gbar, geo.zgb, z);
  bw.side = zmove(bw.side, geo.zside, z);
  bw.lpart = zmove(bw.lpart, (long long)geo.zlpart, z);
  bw.useps = zmove_bytes(bw.useps, bw.zseps, z);
  bw.seps_out = zmove_bytes(bw.seps_out, bw.zseps, z);
  bw.gT_out = zmove(bw.gT_out, geo.zg, z);
  return bw;
}

template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE,
          bool KEEP = false, bool GT = false>
__global__ __launch_bounds__(kWave* Q) void k_expand_d(
    const float* __restrict__ X, const float* __restrict__ G, float* __restrict__ Y,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    const Acc* __restrict__ Us, int OW, int pitch, BwdArgs bw) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  const BwdArgs bz = bwd_at(bw, geo, z);
  const PlaneSrc<CB> src{zmove(X, geo.zx, z), bz.ybar, c0, (int)geo.plane};
  int bx, by;
  xcd_block(bx, by);
  expand_tile<r, CB, R, Q, S1, KIND, Acc, MODE, true, false, KEEP, GT>(
      zmove(G, geo.zg, z), zmove(Y, geo.zy, z), geo, wp, load_lambda(lam_dev, lam_host), c0,
      zmove_bytes(Us, geo.zu, z), OW, pitch, bz, bx, by, gridDim.x, smem, &src);
}

template <int r, int CB, int R, int Q, bool S1, int KIND, typename Acc, int MODE>
__global__ __launch_bounds__(kWave* Q) void k_expand(
    const float* __restrict__ X, const float* __restrict__ G, float* __restrict__ Y,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    const Acc* __restrict__ Us, int OW, int pitch, BwdArgs bw) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  expand_block<r, CB, R, Q, S1, KIND, Acc, MODE>(
      zmove(X, geo.zx, z), zmove(G, geo.zg, z), zmove(Y, geo.zy, z), geo, wp,
      load_lambda(lam_dev, lam_host), c0, zmove_bytes(Us, geo.zu, z), OW, pitch,
      bwd_at(bw, geo, z), blockIdx.x, blockIdx.y, gridDim.x, smem);
}

// ---------------------------------------------------------------------------
// One launch per pass (forward, stride 1, direct reads, transposed output).
//
// The three kernels of a pass run as the units of one grid, ordered by stage:
// gx*gy reduce units first, strip group by strip group (each XCD takes a
// contiguous range of groups), then the expand units.  The last `nlast`
// reduce units of a strip group to finish solve the group's separator
// systems (one wave per strip, the block cyclic reduction of
// k_interface_pcr), while the units of later groups are still reducing.  An
// expand unit waits until the interfaces of the one or two groups its strips
// belong to are solved.  Every wait is on units that precede the waiter in
// the grid: workgroups start in order, so each waited-for unit has started,
// and a waiting last finisher only waits for its own group's reduce units;
// the host admits the launch only while those waiters fill at most half of
// one XCD's resident workgroups.  Waits are bounded (the error word is set
// and the wait abandoned past the spin limit).  Contributions and separators
// pass between workgroups through the device-coherent level (ld / st with
// COH), with no cache-wide fence.
//
// Counters (workspace, zeroed before the launch): red[z * gx + g] counts the
// reduce units of group g of image z that have written their contributions,
// ifc[z * gx + g] the interface units that have written its separators.
// Block 0 of image 0 zeroes the other bank, which the next pass uses.
struct OneSync {
  unsigned int* red;
  unsigned int* ifc;
  unsigned int* next;    // the other bank (nzero words)
  int nzero;
  unsigned int* err;     // kSyncErrMagic after a wait gave up
  unsigned int limit;    // polls per wait before giving up
};

// One lane polls until *c >= target (bounded); no fence: the data it guards
// is read through the coherent level afterwards.
DEV void wait_count(const unsigned int* c, unsigned int target, const OneSync& os) {
  unsigned int it = 0;
  while (__hip_atomic_load(const_cast<unsigned int*>(c), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++it > os.limit) {
      __hip_atomic_store(os.err, kSyncErrMagic, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(16);
  }
}

template <int r, int CB, int R, int Q, int KIND, typename Acc, int MM, bool EXPAND>
__global__ __launch_bounds__(kWave* Q) void k_pass_one(
    const float* __restrict__ X, const float* __restrict__ G, float* __restrict__ Y,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    Acc* __restrict__ sum, Acc* __restrict__ Us, int OW, int pitch, int gx, int gy, int ex,
    int nlast, OneSync os) {
  extern __shared__ float smem[];
  const int z = blockIdx.z;
  if (blockIdx.x == 0 && z == 0)
    for (int i = threadIdx.x; i < os.nzero; i += kWave * Q) os.next[i] = 0u;
  const float lam = load_lambda(lam_dev, lam_host);
  const float* Xz = zmove(X, geo.zx, z);
  const float* Gz = zmove(G, geo.zg, z);
  Acc* sumz = zmove_bytes(sum, geo.zi, z);
  Acc* Usz = zmove_bytes(Us, geo.zu, z);
  const PlaneSrc<CB> src{Xz, nullptr, c0, (int)geo.plane};
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nred = geo.P > 1 ? gx * gy : 0;
  __shared__ unsigned int ticket;
  if ((int)blockIdx.x < nred) {
    const int logical = xcd_rank(blockIdx.x, nred);
    const int bx = logical / gy, by = logical - bx * gy;   // group-major
    reduce_tile<r, CB, R, Q, true, KIND, Acc, kModeForward, true, true>(
        geo, wp, lam, 0, sumz, bx, by, smem, Gz, &src);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's contributions are stored
    __syncthreads();
    unsigned int* red = os.red + ((size_t)z * gx + bx) * kCounterStride;
    if (threadIdx.x == 0)
      ticket = __hip_atomic_fetch_add(red, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = (int)ticket - (gy - nlast);
    if (t < 0) return;
    // one of the group's last nlast units: the separator systems of its strips
    if (threadIdx.x == 0) wait_count(red, (unsigned int)gy, os);
    __syncthreads();
    const int k0 = bx * kWave, nstr = min(kWave, geo.nK - k0);
    const int m = (geo.P - 1 + kWave - 1) / kWave;
    for (int l = t * Q + wq; l < nstr; l += nlast * Q)
      iface_pcr_strip<r, CB, MM, Acc, true>(sumz, Usz, geo.P, m, k0 + l);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's separators are stored
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(os.ifc + ((size_t)z * gx + bx) * kCounterStride, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  if constexpr (EXPAND) {
  const int e = blockIdx.x - nred;
  const int logical = xcd_rank(e, ex * gy);
  const int bx = logical / gy, by = logical - bx * gy;     // group-major
  if (geo.P > 1 && threadIdx.x == 0) {
    const int ki_lo = expand_first_strip(bx, OW, geo, r);
    const int ki_hi = min(ki_lo + kWave - 1, geo.nK - 1);
    wait_count(os.ifc + ((size_t)z * gx + ki_lo / kWave) * kCounterStride, (unsigned int)nlast, os);
    wait_count(os.ifc + ((size_t)z * gx + ki_hi / kWave) * kCounterStride, (unsigned int)nlast, os);
  }
  __syncthreads();
  const BwdArgs none{};
  expand_tile<r, CB, R, Q, true, KIND, Acc, kModeForward, true, true>(
      Gz, zmove(Y, geo.zy, z), geo, wp, lam, c0, Usz, OW, pitch, none, bx, by, ex, smem, &src);
  }
}

// ---------------------------------------------------------------------------
// Launch of one pass for one (r, channel block, precision, stride class,
// weight kind, variant, mode).
template <int r, int CB, int fp64, bool S1, int KIND, int R, int Q, int MODE, int D = 0>
hipError_t launch_impl(const float* x, const float* g, float* y, int c0, const PassGeom& geo,
                       const PassPlan& pl, const WeightParams& wp, const float* lam_dev,
                       float lam_host, void* iface, hipStream_t stream, int stages,
                       const BwdArgs& bw) {
  using Acc = typename std::conditional<fp64 != 0, double, float>::type;
  constexpr int NR = MODE == kModeBackward ? 2 * CB : CB;
  constexpr VariantSet VS = variants_for(MODE, r, CB, fp64);
  using LY = IfaceLayout<r, NR>;
  Acc* sum = reinterpret_cast<Acc*>(iface);
  Acc* us = pl.us_out ? reinterpret_cast<Acc*>(pl.us_out) : sum + pl.sum_elems;
  Acc* gb = sum + pl.sum_elems + pl.u_elems;
  const size_t tile = sizeof(float) * (size_t)(NR + 1) * (Q * R + 2) * pl.pitch;
  const size_t stage_out = sizeof(Acc) * (size_t)kWave * Q * LY::F;
  const int gy = (geo.P + Q - 1) / Q;
  const int nz = geo.nimg > 0 ? geo.nimg : 1;   // images of an NCHW batch (blockIdx.z)
  if constexpr (D != 0 && S1 && MODE == kModeForward && VS.MM > 0) {
    if (pl.one && geo.sb == 1 && geo.out_t && stages == kStageAll && geo.P > 1 &&
        pl.iface_m > 0 && pl.iface_m <= VS.MM) {
      constexpr int MM = VS.MM;
      const bool full = pl.one->full;
      auto kern = full ? k_pass_one<r, CB, R, Q, KIND, Acc, MM, true>
                       : k_pass_one<r, CB, R, Q, KIND, Acc, MM, false>;
      const int gx = (geo.nK + kWave - 1) / kWave;
      const int ex = (geo.W + pl.OW - 1) / pl.OW;
      const int nlast = std::min(gy, (kWave + Q - 1) / Q);
      const size_t lds = std::max(stage_out, sizeof(float) * CB * Q * R * (kWave + 1));
      static int per_cu_of[2] = {-1, -1};   // resident workgroups per CU of each form
      int& per_cu = per_cu_of[full ? 1 : 0];
      if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kern),
                                                         kWave * Q, lds) != hipSuccess) {
          (void)hipGetLastError();
          nb = 0;
        }
        per_cu = nb;
      }
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 0;
      }
      // Waiting last finishers take at most half of one XCD's resident
      // workgroups, and the counters fit their bank.
      if (2LL * nlast * 8 <= (long long)per_cu * cus && (long long)nz * gx <= pl.one->counters) {
        OneCtl& ctl = *pl.one;
        if (!ctl.zeroed[ctl.bank]) {
          const hipError_t e = launch_zero_words(ctl.bank_ptr(ctl.bank), ctl.bank_words(), stream);
          if (e != hipSuccess) return e;
        }
        OneSync os{ctl.bank_ptr(ctl.bank), ctl.bank_ptr(ctl.bank) + ctl.counters * kCounterStride,
                   ctl.bank_ptr(1 - ctl.bank), ctl.bank_words(), ctl.err, ctl.limit};
        ctl.zeroed[1 - ctl.bank] = true;   // this launch zeroes the other bank
        ctl.zeroed[ctl.bank] = false;
        ctl.bank = 1 - ctl.bank;
        const int nred = gx * gy;
        hipLaunchKernelGGL(kern, dim3(nred + (full ? ex * gy : 0), 1, nz), dim3(kWave * Q),
                           full ? lds : stage_out, stream, x, g, y, geo, wp, lam_dev, lam_host, c0,
                           sum, us, pl.OW, pl.pitch, gx, gy, ex, nlast, os);
        if (full) return hipGetLastError();
        stages = kStageExpand;   // the separators are solved: expand in a launch of its own
      }
    }
  }
  if (geo.P > 1 && (stages & kStageReduce)) {
    const int gx = (geo.nK + kWave - 1) / kWave;
    bool direct = false;
    if constexpr (D) {
      if (geo.sb == 1) {
        direct = true;
        hipLaunchKernelGGL((k_reduce_d<r, CB, R, Q, S1, KIND, Acc, MODE>), dim3(gx, gy, nz),
                           dim3(kWave * Q), stage_out, stream, x, bw.ybar, g, geo, wp, lam_dev,
                           lam_host, c0, sum);
      }
    }
    if constexpr (MODE == kModeAdjoint) {
      if (!direct) return hipErrorInvalidValue;   // direct stride-1 chunks only
    } else if (!direct) {
      hipLaunchKernelGGL((k_reduce<r, CB, R, Q, S1, KIND, Acc, MODE>), dim3(gx, gy, nz),
                         dim3(kWave * Q), std::max(tile, stage_out), stream, x, bw.ybar, g, geo,
                         wp, lam_dev, lam_host, c0, pl.pitch, sum);
    }
  }
  if (geo.P > 1 && (stages & kStageInterface)) {
    if (VS.MM > 0 && pl.iface_m > 0 && pl.iface_m <= VS.MM) {
      constexpr int MM = VS.MM > 0 ? VS.MM : 1;
      hipLaunchKernelGGL((k_interface_pcr<r, NR, MM, Acc>), dim3(geo.nK, 1, nz), dim3(kWave), 0,
                         stream, (const Acc*)sum, us, geo.nK, geo.P, pl.iface_m, geo.zi, geo.zu);
    } else if (pl.mw_nl > 0) {
      if constexpr (r == 3 && fp64 == 0 && MODE == kModeForward) {
        const int nl = pl.mw_nl;
        const int m = (geo.P - 1 + nl - 1) / nl;
        const size_t xs = sizeof(Acc) * (size_t)nl * kMwSlot<r, NR>;
        if (nl == 4 * kWave)
          hipLaunchKernelGGL((k_interface_pcr_mw<r, NR, Acc, 4 * kWave>), dim3(geo.nK, 1, nz),
                             dim3(nl), xs, stream, (const Acc*)sum, us, geo.P, m, geo.zi, geo.zu);
        else
          hipLaunchKernelGGL((k_interface_pcr_mw<r, NR, Acc, 2 * kWave>), dim3(geo.nK, 1, nz),
                             dim3(nl), xs, stream, (const Acc*)sum, us, geo.P, m, geo.zi, geo.zu);
      } else {
        return hipErrorInvalidValue;
      }
    } else {
      // Runs longer than the register solver holds: the same wave solver with
      // its per-block values in the scratch part of the interface buffer.
      const int nl = pl.long_nl;
      const int m = (geo.P - 1 + nl - 1) / nl;
      const size_t xs = nl > kWave ? sizeof(Acc) * (size_t)nl * kMwSlot<r, NR> : 0;
      if (nl == 4 * kWave)
        hipLaunchKernelGGL((k_interface_pcr_long<r, NR, Acc, 4 * kWave>), dim3(geo.nK, 1, nz),
                           dim3(nl), xs, stream, (const Acc*)sum, us, gb, geo.P, m, geo.zi, geo.zu);
      else if (nl == 2 * kWave)
        hipLaunchKernelGGL((k_interface_pcr_long<r, NR, Acc, 2 * kWave>), dim3(geo.nK, 1, nz),
                           dim3(nl), xs, stream, (const Acc*)sum, us, gb, geo.P, m, geo.zi, geo.zu);
      else
        hipLaunchKernelGGL((k_interface_pcr_long<r, NR, Acc, kWave>), dim3(geo.nK, 1, nz),
                           dim3(kWave), 0, stream, (const Acc*)sum, us, gb, geo.P, m, geo.zi, geo.zu);
    }
  }
  if constexpr (MODE != kModeAdjoint) {
  if (stages & kStageExpand) {
    const int ex = (geo.W + pl.OW - 1) / pl.OW;
    bool direct = false;
    // Kept separators of the backward's cut: the row-wise stores of the direct
    // stride-1 forward, compiled only where no forward variant is cut like
    // the backward (elsewhere the interface writes them).
    constexpr bool KEEP = MODE == kModeForward && D && S1 && !forward_cut_like_backward(r, CB, fp64);
    if (bw.gT_out) {
      // pass 0 of a filter call: the guidance transposed from the staged tile
      if constexpr (MODE == kModeForward && D && S1) {
        if (geo.sb != 1 || !geo.out_t || bw.seps_out) return hipErrorInvalidValue;
        const size_t lds = sizeof(float) * (CB + 1) * Q * R * (kWave + 1);
        hipLaunchKernelGGL((k_expand_d<r, CB, R, Q, S1, KIND, Acc, MODE, false, true>),
                           dim3(ex, gy, nz), dim3(kWave * Q), lds, stream, x, g, y, geo, wp,
                           lam_dev, lam_host, c0, (const Acc*)us, pl.OW, pl.pitch, bw);
        return hipGetLastError();
      } else {
        return hipErrorInvalidValue;
      }
    }
    if (bw.seps_out) {
      if constexpr (KEEP) {
        if (geo.sb != 1) return hipErrorInvalidValue;
        const size_t lds = geo.out_t ? sizeof(float) * CB * Q * R * (kWave + 1) : 0;
        hipLaunchKernelGGL((k_expand_d<r, CB, R, Q, S1, KIND, Acc, MODE, true>), dim3(ex, gy, nz),
                           dim3(kWave * Q), lds, stream, x, g, y, geo, wp, lam_dev, lam_host, c0,
                           (const Acc*)us, pl.OW, pl.pitch, bw);
        return hipGetLastError();
      } else {
        return hipErrorInvalidValue;
      }
    }
    if constexpr (D) {
      if (geo.sb == 1) {
        // Stride 1: LDS only to stage a transposed store.  Strided: LDS
        // accumulator planes for the covering strips (one per output plane).
        constexpr int NO = MODE == kModeBackward ? CB + 1 : CB;
        const size_t lds = S1 ? (geo.out_t ? sizeof(float) * CB * Q * R * (kWave + 1) : 0)
                              : sizeof(float) * (size_t)NO * (Q * R + 2) * pl.pitch;
        direct = true;
        hipLaunchKernelGGL((k_expand_d<r, CB, R, Q, S1, KIND, Acc, MODE>), dim3(ex, gy, nz),
                           dim3(kWave * Q), lds, stream, x, g, y, geo, wp, lam_dev, lam_host, c0,
                           (const Acc*)us, pl.OW, pl.pitch, bw);
      }
    }
    if (!direct) {
      if (geo.out_t) return hipErrorInvalidValue;   // needs the direct forward kernels
      hipLaunchKernelGGL((k_expand<r, CB, R, Q, S1, KIND, Acc, MODE>), dim3(ex, gy, nz),
                         dim3(kWave * Q), tile, stream, x, g, y, geo, wp, lam_dev, lam_host, c0,
                         (const Acc*)us, pl.OW, pl.pitch, bw);
    }
  }
  }
  return hipGetLastError();
}

// Runtime selection of the compiled variant (stride-1 passes) or of the
// strided kernel (variant 0's R, one chunk per block).
template <int r, int CB, int fp64, int KIND, int MODE, int VI>
hipError_t launch_variant(int vi, const float* x, const float* g, float* y, int c0,
                          const PassGeom& geo, const PassPlan& pl, const WeightParams& wp,
                          const float* lam_dev, float lam_host, void* iface, hipStream_t s,
                          int st, const BwdArgs& bw) {
  constexpr VariantSet VS = variants_for(MODE, r, CB, fp64);
  if constexpr (VI < VS.n) {
    if (vi == VI)
      return launch_impl<r, CB, fp64, true, KIND, VS.v[VI].R, VS.v[VI].Q, MODE, VS.v[VI].D>(
          x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw);
    return launch_variant<r, CB, fp64, KIND, MODE, VI + 1>(vi, x, g, y, c0, geo, pl, wp, lam_dev,
                                                           lam_host, iface, s, st, bw);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int r, int CB, int fp64, int KIND, int MODE>
hipError_t launch_kind(const float* x, const float* g, float* y, int c0, const PassGeom& geo,
                       const PassPlan& pl, const WeightParams& wp, const float* lam_dev,
                       float lam_host, void* iface, hipStream_t s, int st, const BwdArgs& bw) {
  constexpr VariantSet VS = variants_for(MODE, r, CB, fp64);
  if constexpr (MODE == kModeAdjoint) {
    if (geo.stride != 1) return hipErrorInvalidValue;   // stride-1 frames only
  } else if (geo.stride != 1) {
    // Strided forward column passes read their chunks directly (no input tile).
    if constexpr (MODE == kModeForward) {
      constexpr StridedVariant S1v = strided_variant(r, CB, fp64, 1);
      if (pl.variant == 1)
        return launch_impl<r, CB, fp64, false, KIND, S1v.R, S1v.Q, MODE, 1>(
            x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw);
      constexpr int RH = strided_half_R(r, CB, fp64);
      if constexpr (RH > 0) {
        constexpr StridedVariant S2v = strided_variant(r, CB, fp64, 2);
        if (pl.variant == 2)
          return launch_impl<r, CB, fp64, false, KIND, S2v.R, S2v.Q, MODE, 1>(
              x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw);
      }
    }
    return launch_impl<r, CB, fp64, false, KIND, VS.v[0].R, 1, MODE,
                       MODE == kModeForward ? 1 : 0>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                                     iface, s, st, bw);
  }
  return launch_variant<r, CB, fp64, KIND, MODE, 0>(pl.variant, x, g, y, c0, geo, pl, wp,
                                                    lam_dev, lam_host, iface, s, st, bw);
}

template <int r, int CB, int fp64, int MODE>
hipError_t launch_prec(const float* x, const float* g, float* y, int c0, const PassGeom& geo,
                       const PassPlan& pl, const WeightParams& wp, const float* lam_dev,
                       float lam_host, void* iface, hipStream_t s, int st, const BwdArgs& bw) {
  return wp.kind == 0
             ? launch_kind<r, CB, fp64, 0, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                                 iface, s, st, bw)
             : launch_kind<r, CB, fp64, 1, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                                 iface, s, st, bw);
}

template <int r, int MODE>
hipError_t launch_mode(int cb, int fp64, const float* x, const float* g, float* y, int c0,
                       const PassGeom& geo, const PassPlan& pl, const WeightParams& wp,
                       const float* lam_dev, float lam_host, void* iface, hipStream_t s, int st,
                       const BwdArgs& bw) {
  if (cb == 3)
    return fp64 ? launch_prec<r, 3, 1, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw)
                : launch_prec<r, 3, 0, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw);
  return fp64 ? launch_prec<r, 1, 1, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw)
              : launch_prec<r, 1, 0, MODE>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st, bw);
}

template <int r>
hipError_t launch_r(int cb, int fp64, const float* x, const float* g, float* y, int c0,
                    const PassGeom& geo, const PassPlan& pl, const WeightParams& wp,
                    const float* lam_dev, float lam_host, void* iface, hipStream_t s, int st,
                    const BwdArgs* bw) {
  if (pl.mode == kModeBackward)
    return launch_mode<r, kModeBackward>(cb, fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                         iface, s, st, *bw);
  const BwdArgs none{};
  if (pl.mode == kModeForward && bw)   // a forward that keeps separators
    return launch_mode<r, kModeForward>(cb, fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                        iface, s, st, *bw);
  if (pl.mode == kModeAdjoint)
    return launch_mode<r, kModeAdjoint>(cb, fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                        iface, s, st, none);
  return launch_mode<r, kModeForward>(cb, fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host,
                                      iface, s, st, none);
}

}  // namespace

// Defines launch_pass_r<RR> in the translation unit that instantiates radius RR.
#define SGWLS_DEFINE_LAUNCH(RR)                                                              \
  hipError_t launch_pass_r##RR(int cb, int fp64, const float* x, const float* g, float* y,  \
                               int c0, const PassGeom& geo, const PassPlan& plan,           \
                               const WeightParams& wp, const float* lam_dev,                \
                               float lam_host, void* iface, hipStream_t stream, int stages, \
                               const BwdArgs* bw) {                                          \
    return launch_r<RR>(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface,     \
                        stream, stages, bw);                                                 \
  }

}  // namespace sgwls
