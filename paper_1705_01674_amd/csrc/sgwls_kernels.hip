// HIP kernels for one SG-WLS pass on gfx950 (MI355X).
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
// complement) method:
//
//   k_reduce    one lane per (strip, chunk): the last r elements of every
//               chunk but the last are a separator block S_j.  The lane
//               eliminates its chunk's interior I_j (banded LDL^T, right-looking
//               (r+1)x(r+1) window) while carrying the previous separator
//               S_{j-1} as a border; the result is the chunk's contribution to
//               the Schur complement on the separators: the blocks
//               A_{SS} - A_{S I} A_I^{-1} A_{I S} and the matching RHS terms.
//   k_interface one lane per strip: block-tridiagonal (r x r blocks) Cholesky
//               solve of the separator system, one block per chunk boundary.
//   k_expand    one wave per (64 strips, chunk): each lane re-solves its
//               chunk interior with both separators known (they move to the
//               right-hand side), back-substitutes, and the wave averages the
//               strips covering each pixel in LDS in a fixed order (no
//               atomics, bitwise reproducible), then writes its owned pixels.
//
// The weights and the band of A_s are recomputed from the guidance in every
// kernel; nothing of size O(pixels) is stored besides the output.
// Lanes of a wave are adjacent strips, so in the column pass consecutive lanes
// read consecutive pixels of a row.
#include "sgwls_internal.hpp"

#include <algorithm>

namespace sgwls {
namespace {

#define DEV __device__ __forceinline__

// Range factor of Eq. (2).  exp: exp(-dG^2 / (2 sigma_r^2)); frac:
// 1 / (|dG|^alpha_r + eps).  The spatial factor is folded into lambda*S(d).
DEV float range_weight(float dg, const WeightParams& wp) {
  if (wp.kind == 0) return expf(-(dg * dg) * wp.range_c);
  const float ad = fabsf(dg);
  const float pw = (wp.alpha_r == 0.0f) ? 1.0f : (ad > 0.0f ? powf(ad, wp.alpha_r) : 0.0f);
  return 1.0f / (pw + wp.eps);
}

// Element m of a chunk (local index; negative = the previous chunk's tail)
// lies in chunk row floor(m / (2r+1)) at position q = m mod (2r+1).  Chunks
// start on even subsystem rows (R is even), so a row's parity is that of its
// local row index: even rows run k-r..k+r, odd rows k+r..k-r (Sec. 2.1 with
// 1-based rows, where the even ones are reversed).
template <int r>
DEV constexpr int row_of(int m) {
  return m >= 0 ? m / (2 * r + 1) : -1 - ((-m - 1) / (2 * r + 1));
}

template <int r, int R>
struct Chunk {
  static constexpr int w = 2 * r + 1;
  static constexpr int E = R * w;          // elements per full chunk
  static_assert(R >= 2 && R % 2 == 0, "chunks must start on even rows");
  long long base;                          // offset of pixel (a0, k)
  long long sa, sb;
  int a0, L;
  DEV long long off(int m) const {
    const int rho = row_of<r>(m);
    const int q = m - rho * w;
    const int db = (rho & 1) ? (r - q) : (q - r);
    return base + (long long)rho * sa + (long long)db * sb;
  }
  DEV bool ok(int m) const {
    const int a = a0 + row_of<r>(m);
    return a >= 0 && a < L;
  }
};

// lambda * w(m, m+d) for local m in [-r, E) and d = 1..r, at lw[m + r][d - 1];
// zero where either end lies outside the subsystem.
template <int r, int R>
DEV void chunk_weights(const Chunk<r, R>& ch, const float* __restrict__ G,
                       const WeightParams& wp, const float (&lamS)[r + 1],
                       float (&lw)[Chunk<r, R>::E + r][r]) {
  constexpr int E = Chunk<r, R>::E;
  float gv[E + 2 * r];
  bool okv[E + 2 * r];
#pragma unroll
  for (int m = -r; m < E + r; ++m) {
    okv[m + r] = ch.ok(m);
    gv[m + r] = okv[m + r] ? G[ch.off(m)] : 0.0f;
  }
#pragma unroll
  for (int m = -r; m < E; ++m) {
#pragma unroll
    for (int d = 1; d <= r; ++d) {
      lw[m + r][d - 1] = (okv[m + r] && okv[m + d + r])
                             ? lamS[d] * range_weight(gv[m + r] - gv[m + d + r], wp)
                             : 0.0f;
    }
  }
}

// Diagonal of A_s at local element m: 1 + lambda * (sum of its edge weights).
template <int r, int R, typename Acc>
DEV Acc diag_at(const float (&lw)[Chunk<r, R>::E + r][r], int m) {
  Acc s = Acc(1);
#pragma unroll
  for (int d = 1; d <= r; ++d) s += Acc(lw[m + r][d - 1]) + Acc(lw[m - d + r][d - 1]);
  return s;
}

template <typename Acc> DEV Acc rcp_exact(Acc x) { return Acc(1) / x; }

// In-place Cholesky of a small SPD matrix (lower triangle used) and solves.
template <int n, typename Acc>
DEV void chol(Acc (&A)[n][n]) {
#pragma unroll
  for (int j = 0; j < n; ++j) {
    Acc d = A[j][j];
#pragma unroll
    for (int t = 0; t < j; ++t) d -= A[j][t] * A[j][t];
    d = sqrt(d);
    A[j][j] = d;
    const Acc inv = Acc(1) / d;
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
#pragma unroll
  for (int c = 0; c < m; ++c) {
#pragma unroll
    for (int i = 0; i < n; ++i) {
      Acc v = B[i][c];
#pragma unroll
      for (int t = 0; t < i; ++t) v -= Lc[i][t] * B[t][c];
      B[i][c] = v / Lc[i][i];
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
      Acc v = B[i][c];
#pragma unroll
      for (int t = i + 1; t < n; ++t) v -= Lc[t][i] * B[t][c];
      B[i][c] = v / Lc[i][i];
    }
  }
}

template <int r, int CB>
struct IfaceLayout {
  static constexpr int T2 = r * (r + 1) / 2;
  static constexpr int oW = 0;                  // A_SS - A_SI A_I^-1 A_IS of S_j (lower)
  static constexpr int oRf = T2;                // f_S - A_SI A_I^-1 f_I of S_j
  static constexpr int oTT = T2 + r * CB;       // A_TI A_I^-1 A_IT of T = S_{j-1} (lower)
  static constexpr int oRT = 2 * T2 + r * CB;   // A_TI A_I^-1 f_I
  static constexpr int oTB = 2 * T2 + 2 * r * CB;  // coupling S_j <-> S_{j-1} after elimination
  static constexpr int F = 2 * T2 + 2 * r * CB + r * r;
};

DEV float load_lambda(const float* lam_dev, float lam_host) {
  return lam_dev ? *lam_dev : lam_host;
}

// ---------------------------------------------------------------------------
// k_reduce: Schur complement contributions of one chunk of one subsystem.
template <int r, int CB, int R, typename Acc>
__global__ __launch_bounds__(kWave) void k_reduce(
    const float* __restrict__ X, const float* __restrict__ G, PassGeom geo, WeightParams wp,
    const float* __restrict__ lam_dev, float lam_host, int c0, Acc* __restrict__ sum) {
  using CK = Chunk<r, R>;
  using LY = IfaceLayout<r, CB>;
  constexpr int E = CK::E;
  const int ki = blockIdx.x * kWave + threadIdx.x;
  const int j = blockIdx.y;
  if (ki >= geo.nK) return;
  const float lam = load_lambda(lam_dev, lam_host);
  float lamS[r + 1];
#pragma unroll
  for (int d = 0; d <= r; ++d) lamS[d] = lam * wp.spatial[d];
  const int k = min(r + ki * geo.stride, geo.W - 1 - r);
  CK ch;
  ch.a0 = j * R;
  ch.L = geo.L;
  ch.sa = geo.sa;
  ch.sb = geo.sb;
  ch.base = (long long)ch.a0 * geo.sa + (long long)k * geo.sb;
  const bool hasT = j > 0, hasB = j + 1 < geo.P;
  float lw[E + r][r];
  chunk_weights<r, R>(ch, G, wp, lamS, lw);
  const float* Xc = X + (long long)c0 * geo.plane;
  auto fval = [&](int m, int c) -> Acc {
    return ch.ok(m) ? Acc(Xc[(long long)c * geo.plane + ch.off(m)]) : Acc(0);
  };

  Acc W[r + 1][r + 1];   // Schur complement on the window, lower triangle
  Acc Bt[r + 1][r];      // window couplings to the previous separator
  Acc Rw[r + 1][CB];     // window right-hand sides
  Acc TT[r][r], RT[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a) {
#pragma unroll
    for (int b = 0; b < r; ++b) TT[a][b] = Acc(0);
#pragma unroll
    for (int c = 0; c < CB; ++c) RT[a][c] = Acc(0);
  }
#pragma unroll
  for (int a = 0; a < r; ++a) {
    W[a][a] = diag_at<r, R, Acc>(lw, a);
#pragma unroll
    for (int b = 0; b < a; ++b) W[a][b] = -Acc(lw[b + r][a - b - 1]);
#pragma unroll
    for (int c = 0; c < r; ++c) Bt[a][c] = (c >= a) ? -Acc(lw[c][a + r - c - 1]) : Acc(0);
#pragma unroll
    for (int c = 0; c < CB; ++c) Rw[a][c] = fval(a, c);
  }

  auto step = [&](const int m) {
    const int n = m + r;                 // element entering the window
    if (n < E) {
      W[r][r] = diag_at<r, R, Acc>(lw, n);
#pragma unroll
      for (int b = 0; b < r; ++b) W[r][b] = -Acc(lw[m + b + r][r - b - 1]);
#pragma unroll
      for (int c = 0; c < CB; ++c) Rw[r][c] = fval(n, c);
    } else {                             // past the end of the subsystem
      W[r][r] = Acc(1);
#pragma unroll
      for (int b = 0; b < r; ++b) W[r][b] = Acc(0);
#pragma unroll
      for (int c = 0; c < CB; ++c) Rw[r][c] = Acc(0);
    }
#pragma unroll
    for (int c = 0; c < r; ++c) Bt[r][c] = Acc(0);

    const Acc invD = rcp_exact(W[0][0]);
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
      for (int h = 0; h < CB; ++h) RT[c][h] += bs * Rw[0][h];
    }
#pragma unroll
    for (int a = 1; a <= r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) Rw[a][h] -= l[a] * Rw[0][h];
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int b = 0; b <= a; ++b) W[a][b] = W[a + 1][b + 1];
#pragma unroll
      for (int c = 0; c < r; ++c) Bt[a][c] = Bt[a + 1][c];
#pragma unroll
      for (int h = 0; h < CB; ++h) Rw[a][h] = Rw[a + 1][h];
    }
  };
  // Interior elements of a chunk with a separator: 0..E-r-1.  The last chunk
  // has no separator and eliminates all E (padding past the end is inert).
#pragma unroll
  for (int m = 0; m < E - r; ++m) step(m);
  if (!hasB) {
#pragma unroll
    for (int m = E - r; m < E; ++m) step(m);
  }

  Acc* out = sum + (size_t)j * LY::F * geo.nK + ki;
  const size_t fs = geo.nK;
  if (hasB) {
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) out[(LY::oW + t++) * fs] = W[a][b];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) out[(LY::oRf + a * CB + h) * fs] = Rw[a][h];
  }
  if (hasT) {
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) out[(LY::oTT + t++) * fs] = TT[a][b];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) out[(LY::oRT + a * CB + h) * fs] = RT[a][h];
  }
  if (hasT && hasB) {
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int c = 0; c < r; ++c) out[(LY::oTB + a * r + c) * fs] = Bt[a][c];
  }
}

// ---------------------------------------------------------------------------
// k_interface: block-tridiagonal separator system of one subsystem.
// Sigma_jj = W_j - TT_{j+1},  Sigma_{j,j+1}[a][c] = TB_{j+1}[c][a],
// rhs_j = Rf_j - RT_{j+1};  block Cholesky forward sweep, then back sweep.
// U receives u on every separator: U[(j*r*CB + a*CB + h) * nK + ki].
template <int r, int CB, typename Acc>
__global__ __launch_bounds__(kWave) void k_interface(const Acc* __restrict__ sum,
                                                     Acc* __restrict__ Gb, Acc* __restrict__ U,
                                                     int nK, int P) {
  using LY = IfaceLayout<r, CB>;
  const int ki = blockIdx.x * kWave + threadIdx.x;
  if (ki >= nK) return;
  auto S = [&](int j, int f) -> Acc { return sum[((size_t)j * LY::F + f) * nK + ki]; };
  Acc Gp[r][r], hp[r][CB];
#pragma unroll
  for (int a = 0; a < r; ++a) {
#pragma unroll
    for (int b = 0; b < r; ++b) Gp[a][b] = Acc(0);
#pragma unroll
    for (int h = 0; h < CB; ++h) hp[a][h] = Acc(0);
  }
  for (int j = 0; j < P - 1; ++j) {
    Acc A[r][r], y[r][CB];
    int t = 0;
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        A[a][b] = S(j, LY::oW + t) - S(j + 1, LY::oTT + t);
        A[b][a] = A[a][b];
        ++t;
      }
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h)
        y[a][h] = S(j, LY::oRf + a * CB + h) - S(j + 1, LY::oRT + a * CB + h);
    if (j > 0) {
      Acc Up[r][r];   // Sigma_{j-1,j}
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Up[a][c] = S(j, LY::oTB + c * r + a);
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int b = 0; b < r; ++b) {
          Acc v = A[a][b];
#pragma unroll
          for (int c = 0; c < r; ++c) v -= Up[c][a] * Gp[c][b];
          A[a][b] = v;
        }
#pragma unroll
        for (int h = 0; h < CB; ++h) {
          Acc v = y[a][h];
#pragma unroll
          for (int c = 0; c < r; ++c) v -= Up[c][a] * hp[c][h];
          y[a][h] = v;
        }
      }
    }
    chol<r, Acc>(A);
    Acc Gn[r][r];
    if (j + 1 < P - 1) {
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Gn[a][c] = S(j + 1, LY::oTB + c * r + a);
      chol_solve<r, r, Acc>(A, Gn);
    } else {
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int c = 0; c < r; ++c) Gn[a][c] = Acc(0);
    }
    chol_solve<r, CB, Acc>(A, y);
#pragma unroll
    for (int a = 0; a < r; ++a) {
#pragma unroll
      for (int c = 0; c < r; ++c) {
        Gb[((size_t)j * r * r + a * r + c) * nK + ki] = Gn[a][c];
        Gp[a][c] = Gn[a][c];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        U[((size_t)j * r * CB + a * CB + h) * nK + ki] = y[a][h];
        hp[a][h] = y[a][h];
      }
    }
  }
  for (int j = P - 3; j >= 0; --j) {
    Acc u[r][CB];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        Acc v = U[((size_t)j * r * CB + a * CB + h) * nK + ki];
#pragma unroll
        for (int c = 0; c < r; ++c) v -= Gb[((size_t)j * r * r + a * r + c) * nK + ki] * hp[c][h];
        u[a][h] = v;
      }
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        U[((size_t)j * r * CB + a * CB + h) * nK + ki] = u[a][h];
        hp[a][h] = u[a][h];
      }
  }
}

// ---------------------------------------------------------------------------
// k_expand: final solve of every chunk with its separators known, scatter and
// average.  Block x owns output columns [x*OW, x*OW + OW) of the pass; its
// 64 lanes are the strips whose 2r+1 columns touch them.
template <int r, int CB, int R, typename Acc>
__global__ __launch_bounds__(kWave) void k_expand(
    const float* __restrict__ X, const float* __restrict__ G, float* __restrict__ Y,
    PassGeom geo, WeightParams wp, const float* __restrict__ lam_dev, float lam_host, int c0,
    const Acc* __restrict__ U, int OW, int accw, int row_major_out) {
  using CK = Chunk<r, R>;
  constexpr int E = CK::E, w = CK::w;
  extern __shared__ float smem[];
  float* acc = smem;                                   // [CB][R][accw]
  int* cnt = reinterpret_cast<int*>(smem + CB * R * accw);   // [accw]
  const int lane = threadIdx.x, j = blockIdx.y;
  const int b_lo = blockIdx.x * OW, b_hi = min(b_lo + OW, geo.W);
  int ki_lo;
  if (geo.stride == 1) {
    ki_lo = max(0, b_lo - 2 * r);
  } else {
    const int t = b_lo - 2 * r;
    ki_lo = t <= 0 ? 0 : (t + geo.stride - 1) / geo.stride;
  }
  ki_lo = min(ki_lo, geo.nK - 1);
  const int colbase = min(r + ki_lo * geo.stride, geo.W - 1 - r) - r;
  const int ki = ki_lo + lane;
  const bool active = ki < geo.nK;
  const int k = active ? min(r + ki * geo.stride, geo.W - 1 - r) : colbase + r;
  for (int i = lane; i < CB * R * accw; i += kWave) acc[i] = 0.0f;
  for (int i = lane; i < accw; i += kWave) cnt[i] = 0;
  __syncthreads();

  const float lam = load_lambda(lam_dev, lam_host);
  float lamS[r + 1];
#pragma unroll
  for (int d = 0; d <= r; ++d) lamS[d] = lam * wp.spatial[d];
  CK ch;
  ch.a0 = j * R;
  ch.L = geo.L;
  ch.sa = geo.sa;
  ch.sb = geo.sb;
  ch.base = (long long)ch.a0 * geo.sa + (long long)k * geo.sb;
  const bool hasT = j > 0, hasB = j + 1 < geo.P;
  const float* Xc = X + (long long)c0 * geo.plane;

  Acc Z[E][CB];     // z = D^{-1} L^{-1} f, overwritten by the solution u
  if (active) {
    float lw[E + r][r];
    chunk_weights<r, R>(ch, G, wp, lamS, lw);
    auto fval = [&](int m, int c) -> Acc {
      return ch.ok(m) ? Acc(Xc[(long long)c * geo.plane + ch.off(m)]) : Acc(0);
    };
    Acc uT[r][CB], uB[r][CB];
#pragma unroll
    for (int a = 0; a < r; ++a)
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        uT[a][h] = hasT ? U[((size_t)(j - 1) * r * CB + a * CB + h) * geo.nK + ki] : Acc(0);
        uB[a][h] = hasB ? U[((size_t)j * r * CB + a * CB + h) * geo.nK + ki] : Acc(0);
      }
    Acc Lf[E][r];   // Lf[m][a-1] = L(m+a, m)
    Acc W[r + 1][r + 1];
    Acc Rw[r + 1][CB];
#pragma unroll
    for (int a = 0; a < r; ++a) {
      W[a][a] = diag_at<r, R, Acc>(lw, a);
#pragma unroll
      for (int b = 0; b < a; ++b) W[a][b] = -Acc(lw[b + r][a - b - 1]);
#pragma unroll
      for (int h = 0; h < CB; ++h) {
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
        // n belongs to the known separator S_j: move its coupling to the RHS.
        const int bi = n - (E - r);
#pragma unroll
        for (int b = 0; b < r; ++b)
#pragma unroll
          for (int h = 0; h < CB; ++h) Rw[b][h] += Acc(lw[m + b + r][r - b - 1]) * uB[bi][h];
      } else if (n < E) {
        dummy = false;
        W[r][r] = diag_at<r, R, Acc>(lw, n);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = -Acc(lw[m + b + r][r - b - 1]);
#pragma unroll
        for (int h = 0; h < CB; ++h) Rw[r][h] = fval(n, h);
      }
      if (dummy) {
        W[r][r] = Acc(1);
#pragma unroll
        for (int b = 0; b < r; ++b) W[r][b] = Acc(0);
#pragma unroll
        for (int h = 0; h < CB; ++h) Rw[r][h] = Acc(0);
      }
      const Acc invD = rcp_exact(W[0][0]);
      Acc l[r + 1];
#pragma unroll
      for (int a = 1; a <= r; ++a) {
        l[a] = W[a][0] * invD;
        Lf[m][a - 1] = l[a];
      }
#pragma unroll
      for (int h = 0; h < CB; ++h) Z[m][h] = Rw[0][h] * invD;
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int b = 1; b <= a; ++b) W[a][b] -= l[a] * W[b][0];
#pragma unroll
      for (int a = 1; a <= r; ++a)
#pragma unroll
        for (int h = 0; h < CB; ++h) Rw[a][h] -= l[a] * Rw[0][h];
#pragma unroll
      for (int a = 0; a < r; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) W[a][b] = W[a + 1][b + 1];
#pragma unroll
        for (int h = 0; h < CB; ++h) Rw[a][h] = Rw[a + 1][h];
      }
    };
#pragma unroll
    for (int m = 0; m < E - r; ++m) step(m);
    if (!hasB) {
#pragma unroll
      for (int m = E - r; m < E; ++m) step(m);
    }
    if (hasB) {
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int h = 0; h < CB; ++h) Z[E - r + a][h] = uB[a][h];
#pragma unroll
      for (int a = 0; a < r; ++a)
#pragma unroll
        for (int t = 0; t < r; ++t) Lf[E - r + a][t] = Acc(0);
    }
    // back substitution u_m = z_m - sum_a L(m+a, m) u_{m+a}
#pragma unroll
    for (int m = E - 1; m >= 0; --m) {
#pragma unroll
      for (int h = 0; h < CB; ++h) {
        Acc v = Z[m][h];
#pragma unroll
        for (int a = 1; a <= r; ++a)
          if (m + a < E) v -= Lf[m][a - 1] * Z[m + a][h];
        Z[m][h] = v;
      }
    }
  }

  // Average over the strips covering each pixel, in a fixed order (q = 0..2r).
  const int rows = min(R, geo.L - ch.a0);
#pragma unroll
  for (int q = 0; q < w; ++q) {
    if (active) {
#pragma unroll
      for (int rho = 0; rho < R; ++rho) {
        if (rho < rows) {
          const int col = ((rho & 1) ? (k + r - q) : (k - r + q)) - colbase;
#pragma unroll
          for (int h = 0; h < CB; ++h) acc[(h * R + rho) * accw + col] += float(Z[rho * w + q][h]);
        }
      }
      cnt[k - r + q - colbase] += 1;
    }
    __syncthreads();
  }
  const int ncols = b_hi - b_lo;
  const int total = rows * ncols;
  float* Yc = Y + (long long)c0 * geo.plane;
  for (int idx = lane; idx < total; idx += kWave) {
    int rho, b;
    if (row_major_out) {
      rho = idx % rows;
      b = b_lo + idx / rows;
    } else {
      rho = idx / ncols;
      b = b_lo + idx % ncols;
    }
    const float inv = 1.0f / float(cnt[b - colbase]);
    const long long o = (long long)(ch.a0 + rho) * geo.sa + (long long)b * geo.sb;
#pragma unroll
    for (int h = 0; h < CB; ++h)
      Yc[(long long)h * geo.plane + o] = acc[(h * R + rho) * accw + (b - colbase)] * inv;
  }
}

// ---------------------------------------------------------------------------
// Rows per chunk: the expand kernel keeps (r + CB) values per element in
// registers, so R shrinks as r and the channel block grow.
constexpr int rows_table(int r, int cb, int fp64) {
  return fp64 ? (r == 1 ? (cb == 1 ? 8 : 4) : (r == 2 ? (cb == 1 ? 4 : 2) : 2))
              : (r == 1 ? (cb == 1 ? 16 : 8)
                        : (r == 2 ? (cb == 1 ? 6 : 4) : (r == 3 ? (cb == 1 ? 4 : 2) : 2)));
}

template <int r, int CB, int fp64>
hipError_t launch_impl(const float* x, const float* g, float* y, int c0, const PassGeom& geo,
                       const PassPlan& pl, const WeightParams& wp, const float* lam_dev,
                       float lam_host, void* iface, hipStream_t stream, int stages) {
  using Acc = typename std::conditional<fp64 != 0, double, float>::type;
  constexpr int R = rows_table(r, CB, fp64);
  Acc* sum = reinterpret_cast<Acc*>(iface);
  Acc* gb = sum + pl.sum_elems;
  Acc* u = gb + pl.g_elems;
  const int gx = (geo.nK + kWave - 1) / kWave;
  if (geo.P > 1 && (stages & kStageReduce))
    hipLaunchKernelGGL((k_reduce<r, CB, R, Acc>), dim3(gx, geo.P), dim3(kWave), 0, stream, x, g,
                       geo, wp, lam_dev, lam_host, c0, sum);
  if (geo.P > 1 && (stages & kStageInterface))
    hipLaunchKernelGGL((k_interface<r, CB, Acc>), dim3(gx), dim3(kWave), 0, stream,
                       (const Acc*)sum, gb, u, geo.nK, geo.P);
  if (stages & kStageExpand) {
    const int ex = (geo.W + pl.OW - 1) / pl.OW;
    const size_t lds = sizeof(float) * ((size_t)CB * R * pl.accw + pl.accw);
    hipLaunchKernelGGL((k_expand<r, CB, R, Acc>), dim3(ex, geo.P), dim3(kWave), lds, stream, x,
                       g, y, geo, wp, lam_dev, lam_host, c0, (const Acc*)u, pl.OW, pl.accw,
                       geo.sa == 1 ? 1 : 0);
  }
  return hipGetLastError();
}

template <int r, int CB>
hipError_t launch_prec(int fp64, const float* x, const float* g, float* y, int c0,
                       const PassGeom& geo, const PassPlan& pl, const WeightParams& wp,
                       const float* lam_dev, float lam_host, void* iface, hipStream_t s,
                       int st) {
  return fp64 ? launch_impl<r, CB, 1>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st)
              : launch_impl<r, CB, 0>(x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st);
}

template <int r>
hipError_t launch_cb(int cb, int fp64, const float* x, const float* g, float* y, int c0,
                     const PassGeom& geo, const PassPlan& pl, const WeightParams& wp,
                     const float* lam_dev, float lam_host, void* iface, hipStream_t s, int st) {
  return cb == 3
             ? launch_prec<r, 3>(fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st)
             : launch_prec<r, 1>(fp64, x, g, y, c0, geo, pl, wp, lam_dev, lam_host, iface, s, st);
}

}  // namespace

int rows_per_chunk(int r, int cb, int fp64) { return rows_table(r, cb, fp64); }

int strip_count(int W, int r, int stride) {
  if (r < 1 || stride < 1 || W < 2 * r + 1) return 0;
  const int span = W - 1 - 2 * r;          // last regular centre offset
  const int regular = span / stride + 1;
  return regular + ((span % stride) != 0 ? 1 : 0);
}

PassPlan make_plan(int L, int W, int r, int cb, int stride, int fp64) {
  PassPlan pl{};
  pl.R = rows_table(r, cb, fp64);
  pl.P = (L + pl.R - 1) / pl.R;
  pl.nK = strip_count(W, r, stride);
  pl.OW = stride == 1 ? kWave - 2 * r : (kWave - 2) * stride - 2 * r;
  pl.accw = stride == 1 ? kWave + 2 * r : (kWave - 1) * stride + 2 * r + 1;
  const int T2 = r * (r + 1) / 2;
  const int F = 2 * T2 + 2 * r * cb + r * r;
  pl.acc_bytes = fp64 ? 8 : 4;
  pl.sum_elems = (size_t)pl.P * F * pl.nK;
  pl.g_elems = (size_t)std::max(pl.P - 1, 1) * r * r * pl.nK;
  pl.u_elems = (size_t)std::max(pl.P - 1, 1) * r * cb * pl.nK;
  return pl;
}

size_t interface_bytes(const PassPlan& pl) {
  return (pl.sum_elems + pl.g_elems + pl.u_elems) * (size_t)pl.acc_bytes + 256;
}

hipError_t launch_pass(int r, int cb, int fp64, const float* x, const float* g, float* y,
                       int c0, const PassGeom& geo, const PassPlan& plan,
                       const WeightParams& wp, const float* lam_dev, float lam_host,
                       void* iface, hipStream_t stream, int st) {
  switch (r) {
    case 1: return launch_cb<1>(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st);
    case 2: return launch_cb<2>(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st);
    case 3: return launch_cb<3>(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st);
    case 4: return launch_cb<4>(cb, fp64, x, g, y, c0, geo, plan, wp, lam_dev, lam_host, iface, stream, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sgwls
