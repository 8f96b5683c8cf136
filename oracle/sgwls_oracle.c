/*
 * Plain double-precision CPU oracle for Semi-Global Weighted Least Squares
 * (SG-WLS) filtering: W. Liu, X. Chen, C. Shen, Z. Liu, J. Yang,
 * "Semi-Global Weighted Least Squares in Image Filtering", ICCV 2017
 * (arXiv 1705.01674).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, header
 * or constant with the GPU library, and the GPU library never calls it.
 *
 * What it computes, step by step, in the order of Sec. 2.3 of the paper:
 *   1. neighbourhood construction of each 1D subsystem (Sec. 2.1),
 *   2. exact solution of each subsystem A_s u = f (Eq. 5), here by a plain
 *      banded LDL^T factorisation -- a different exact algorithm from the
 *      paper's r-band LU (Eqs. 9-20) and from the GPU's partitioned solver,
 *   3. inverse construction (scatter back to pixels),
 *   4. averaging of the pixels covered by several subsystems,
 * performed T times, column direction then row direction (Sec. 2.3).
 * The guidance weights follow Eq. (2); A_s follows Eq. (4) restricted to the
 * one-dimensional 2r+1 neighbourhood of the constructed vector (Sec. 2.2).
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes of the repository):
 *   - |i-j| in the weight is the distance along the constructed 1D vector
 *     (Sec. 2.2 states that the subsystem's neighbourhood is one-dimensional);
 *   - only pairs 0 < |p-q| <= r of the 1D vector are coupled, and A_s is
 *     exactly I + lambda*L as in Eq. (4) (no factor of two);
 *   - rows are 1-based in the paper and even rows are reversed, so with
 *     0-based rows the odd ones run right-to-left;
 *   - strip centres are r, r+stride, ... (0-based) and the centre N-1-r is
 *     always included so every pixel is covered;
 *   - covered pixels are averaged with equal weights;
 *   - the same lambda is used in every pass; one iteration is a column pass
 *     followed by a row pass; the row pass is the column pass of the
 *     transposed image.
 *
 * Gradients (sgwls backward) are not in the paper; they are the adjoint of the
 * steps above: for an SPD A, d/dx of A^{-1}x is A^{-1} itself, and
 * dA/dw_pq = lambda (e_p - e_q)(e_p - e_q)^T.
 *
 * Every function returns 0 on success and a negative code on bad arguments
 * or a non-positive pivot.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double lambda;  /* smoothness weight lambda, Eq. (1) */
  int r;          /* neighbourhood radius: (2r+1)x(2r+1) window, Eq. (1) */
  int iters;      /* T: column+row iterations, Sec. 2.3 */
  int stride;     /* sliding step tau between strip centres, Sec. 2.3 */
  int kind;       /* 0: omega^exp, 1: omega^frac, Eq. (2) */
  double sigma_s, sigma_r;  /* omega^exp constants */
  double alpha_s, alpha_r;  /* omega^frac constants */
  double eps;               /* omega^frac epsilon (the paper uses 1e-4) */
} orc_params;

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_PIVOT = -2, ORC_E_MEM = -3 };

/* Threads of the parallel loops of later calls (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int check_params(const orc_params* p, int M, int N) {
  if (!p) return ORC_E_ARG;
  if (p->r < 1 || p->stride < 1 || p->stride > 2 * p->r + 1) return ORC_E_ARG;
  if (M < 2 * p->r + 1 || N < 2 * p->r + 1) return ORC_E_ARG;
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda)) return ORC_E_ARG;
  if (p->kind == 0 && !(p->sigma_s > 0.0 && p->sigma_r > 0.0)) return ORC_E_ARG;
  if (p->kind == 1 && !(p->eps > 0.0)) return ORC_E_ARG;
  if (p->kind != 0 && p->kind != 1) return ORC_E_ARG;
  return ORC_OK;
}

/* Strip centres along a dimension of length n (Sec. 2.1: k = r+1..N-r in
 * 1-based terms; Sec. 2.3: consecutive centres are `stride` apart).  Writes up
 * to the count into out (if non-NULL) and returns the count. */
int orc_centres(int n, int r, int stride, int* out) {
  if (r < 1 || stride < 1 || n < 2 * r + 1) return ORC_E_ARG;
  int cnt = 0, last = -1;
  for (int k = r; k <= n - 1 - r; k += stride) {
    if (out) out[cnt] = k;
    cnt++;
    last = k;
  }
  if (last != n - 1 - r) {
    if (out) out[cnt] = n - 1 - r;
    cnt++;
  }
  return cnt;
}

/* Pixel of element p of the column-direction vector centred at column k
 * (Sec. 2.1): row i = p / (2r+1); 0-based even rows run left to right over
 * columns k-r..k+r, odd rows right to left. */
void orc_snake_pixel(int k, int r, int p, int* i, int* j) {
  int w = 2 * r + 1;
  int row = p / w, q = p % w;
  *i = row;
  *j = (row % 2 == 0) ? (k - r + q) : (k + r - q);
}

/* Guidance weight of Eq. (2) for two elements d apart on the 1D vector. */
double orc_weight(const orc_params* p, int d, double ga, double gb) {
  double dd = (double)d, dg = ga - gb;
  if (p->kind == 0)
    return exp(-dd * dd / (2.0 * p->sigma_s * p->sigma_s)) *
           exp(-dg * dg / (2.0 * p->sigma_r * p->sigma_r));
  return 1.0 / (pow(dd, p->alpha_s) + p->eps) *
         1.0 / (pow(fabs(dg), p->alpha_r) + p->eps);
}

/* Partial derivative of the weight with respect to its first guidance value
 * ga.  The derivative with respect to gb is the negative of it.  For
 * omega^frac it is taken as 0 where ga == gb. */
double orc_weight_dga(const orc_params* p, int d, double ga, double gb) {
  double dg = ga - gb;
  if (p->kind == 0) {
    double w = orc_weight(p, d, ga, gb);
    return -w * dg / (p->sigma_r * p->sigma_r);
  }
  if (dg == 0.0) return 0.0;
  double dd = (double)d;
  double spatial = 1.0 / (pow(dd, p->alpha_s) + p->eps);
  double ad = fabs(dg);
  double den = pow(ad, p->alpha_r) + p->eps;
  double sgn = dg > 0.0 ? 1.0 : -1.0;
  return -spatial * p->alpha_r * pow(ad, p->alpha_r - 1.0) * sgn / (den * den);
}

/* Assemble the band of A_s (Eq. 4 on the 1D vector, Eq. 5) for the
 * column-direction vector centred at column k of an M x N guidance image g.
 * s = (2r+1) M.  diag[p] = 1 + lambda * sum of the weights of the edges at p;
 * off[p*r + d-1] = A_s(p, p+d) = -lambda * w(p, p+d) (0 past the end).
 * w (nullable) receives the raw weights in the layout of off. */
int orc_strip_band(int M, int N, const double* g, const orc_params* p, int k,
                   double* diag, double* off, double* w) {
  int r = p->r, s = (2 * r + 1) * M;
  for (int q = 0; q < s; ++q) diag[q] = 1.0;
  for (int q = 0; q < s; ++q) {
    int iq, jq;
    orc_snake_pixel(k, r, q, &iq, &jq);
    for (int d = 1; d <= r; ++d) {
      double wv = 0.0;
      if (q + d < s) {
        int ie, je;
        orc_snake_pixel(k, r, q + d, &ie, &je);
        wv = orc_weight(p, d, g[(size_t)iq * N + jq], g[(size_t)ie * N + je]);
        diag[q] += p->lambda * wv;
        diag[q + d] += p->lambda * wv;
      }
      off[(size_t)q * r + d - 1] = -p->lambda * wv;
      if (w) w[(size_t)q * r + d - 1] = wv;
    }
  }
  return ORC_OK;
}

/* Exact solution of a symmetric positive definite band system of size s and
 * half-bandwidth r by LDL^T factorisation (L unit lower triangular):
 *   D_k     = A_kk - sum_j L_kj^2 D_j
 *   L_mk    = (A_mk - sum_j L_mj L_kj D_j) / D_k,   k < m <= k+r
 * then L y = b, z = D^{-1} y, L^T u = z.  rhs is s x nrhs (row-major) and is
 * overwritten with the solution.  Scratch: Lb (s*r) and D (s). */
static int band_ldlt_solve_ws(int s, int r, const double* diag,
                              const double* off, int nrhs, double* rhs,
                              double* Lb, double* D) {
  /* Lb[k*r + t-1] = L(k, k-t) */
  for (size_t q = 0; q < (size_t)s * r; ++q) Lb[q] = 0.0;
  for (int k = 0; k < s; ++k) {
    double dk = diag[k];
    for (int t = 1; t <= r && k - t >= 0; ++t) {
      double l = Lb[(size_t)k * r + t - 1];
      dk -= l * l * D[k - t];
    }
    if (!(dk > 0.0)) return ORC_E_PIVOT;
    D[k] = dk;
    for (int i = 1; i <= r && k + i < s; ++i) {
      int m = k + i;
      double sum = off[(size_t)k * r + i - 1]; /* A(m, k) = A(k, m) */
      for (int j = (m - r > 0 ? m - r : 0); j < k; ++j)
        sum -= Lb[(size_t)m * r + (m - j) - 1] * Lb[(size_t)k * r + (k - j) - 1] * D[j];
      Lb[(size_t)m * r + i - 1] = sum / dk;
    }
  }
  for (int c = 0; c < nrhs; ++c) {
    for (int k = 0; k < s; ++k) {
      double y = rhs[(size_t)k * nrhs + c];
      for (int t = 1; t <= r && k - t >= 0; ++t)
        y -= Lb[(size_t)k * r + t - 1] * rhs[(size_t)(k - t) * nrhs + c];
      rhs[(size_t)k * nrhs + c] = y;
    }
    for (int k = 0; k < s; ++k) rhs[(size_t)k * nrhs + c] /= D[k];
    for (int k = s - 1; k >= 0; --k) {
      double u = rhs[(size_t)k * nrhs + c];
      for (int i = 1; i <= r && k + i < s; ++i)
        u -= Lb[(size_t)(k + i) * r + i - 1] * rhs[(size_t)(k + i) * nrhs + c];
      rhs[(size_t)k * nrhs + c] = u;
    }
  }
  return ORC_OK;
}

int orc_band_solve(int s, int r, const double* diag, const double* off,
                   int nrhs, double* rhs) {
  if (s < 1 || r < 1 || nrhs < 1) return ORC_E_ARG;
  double* Lb = (double*)malloc(sizeof(double) * (size_t)s * r);
  double* D = (double*)malloc(sizeof(double) * (size_t)s);
  if (!Lb || !D) { free(Lb); free(D); return ORC_E_MEM; }
  int rc = band_ldlt_solve_ws(s, r, diag, off, nrhs, rhs, Lb, D);
  free(Lb);
  free(D);
  return rc;
}

/* One column-direction pass (Sec. 2.3, steps 1-4).  X and Y are C x M x N
 * planar; g is M x N.  cnt (nullable, M x N) receives the number of
 * subsystems covering each pixel.  Y must not alias X. */
int orc_col_pass(int C, int M, int N, const double* X, const double* g,
                 double* Y, const orc_params* p, double* cnt) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (C < 1 || !X || !g || !Y) return ORC_E_ARG;
  int r = p->r, s = (2 * r + 1) * M;
  int nK = orc_centres(N, r, p->stride, NULL);
  int* K = (int*)malloc(sizeof(int) * nK);
  double* U = (double*)malloc(sizeof(double) * (size_t)nK * s * C);
  double* cn = (double*)calloc((size_t)M * N, sizeof(double));
  if (!K || !U || !cn) { free(K); free(U); free(cn); return ORC_E_MEM; }
  orc_centres(N, r, p->stride, K);
  int err = 0;
#pragma omp parallel
  {
    double* diag = (double*)malloc(sizeof(double) * s);
    double* off = (double*)malloc(sizeof(double) * (size_t)s * r);
    double* Lb = (double*)malloc(sizeof(double) * (size_t)s * r);
    double* D = (double*)malloc(sizeof(double) * s);
#pragma omp for schedule(static)
    for (int ki = 0; ki < nK; ++ki) {
      int k = K[ki];
      double* u = U + (size_t)ki * s * C;
      orc_strip_band(M, N, g, p, k, diag, off, NULL);
      for (int q = 0; q < s; ++q) {
        int i, j;
        orc_snake_pixel(k, r, q, &i, &j);
        for (int c = 0; c < C; ++c)
          u[(size_t)q * C + c] = X[((size_t)c * M + i) * N + j];
      }
      if (band_ldlt_solve_ws(s, r, diag, off, C, u, Lb, D) != ORC_OK) {
#pragma omp atomic write
        err = 1;
      }
    }
    free(diag); free(off); free(Lb); free(D);
  }
  if (!err) {
    memset(Y, 0, sizeof(double) * (size_t)C * M * N);
    for (int ki = 0; ki < nK; ++ki) {
      const double* u = U + (size_t)ki * s * C;
      for (int q = 0; q < s; ++q) {
        int i, j;
        orc_snake_pixel(K[ki], r, q, &i, &j);
        for (int c = 0; c < C; ++c) Y[((size_t)c * M + i) * N + j] += u[(size_t)q * C + c];
        cn[(size_t)i * N + j] += 1.0;
      }
    }
    for (int c = 0; c < C; ++c)
      for (size_t q = 0; q < (size_t)M * N; ++q) Y[(size_t)c * M * N + q] /= cn[q];
    if (cnt) memcpy(cnt, cn, sizeof(double) * (size_t)M * N);
  }
  free(K); free(U); free(cn);
  return err ? ORC_E_PIVOT : ORC_OK;
}

static void transpose_planes(int C, int M, int N, const double* in, double* out) {
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < N; ++j)
        out[((size_t)c * N + j) * M + i] = in[((size_t)c * M + i) * N + j];
}

/* One row-direction pass: the column pass of the transposed image. */
int orc_row_pass(int C, int M, int N, const double* X, const double* g,
                 double* Y, const orc_params* p, double* cnt) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (C < 1 || !X || !g || !Y) return ORC_E_ARG;
  size_t n = (size_t)C * M * N;
  double* Xt = (double*)calloc(n, sizeof(double));
  double* Yt = (double*)calloc(n, sizeof(double));
  double* gt = (double*)calloc((size_t)M * N, sizeof(double));
  double* ct = cnt ? (double*)malloc(sizeof(double) * (size_t)M * N) : NULL;
  if (!Xt || !Yt || !gt || (cnt && !ct)) { free(Xt); free(Yt); free(gt); free(ct); return ORC_E_MEM; }
  transpose_planes(C, M, N, X, Xt);
  transpose_planes(1, M, N, g, gt);
  rc = orc_col_pass(C, N, M, Xt, gt, Yt, p, ct);
  if (rc == ORC_OK) {
    transpose_planes(C, N, M, Yt, Y);
    if (cnt) transpose_planes(1, N, M, ct, cnt);
  }
  free(Xt); free(Yt); free(gt); free(ct);
  return rc;
}

/* The SG-WLS filter: T iterations of (column pass, row pass), Sec. 2.3.
 * saved (nullable) receives the input of every pass: 2T planes of C*M*N,
 * pass 2t is the column pass of iteration t and pass 2t+1 its row pass. */
int orc_filter(int C, int M, int N, const double* F, const double* g,
               double* U, const orc_params* p, double* saved) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (p->iters < 1 || C < 1 || !F || !g || !U) return ORC_E_ARG;
  size_t n = (size_t)C * M * N;
  double* tmp = (double*)malloc(sizeof(double) * n);
  if (!tmp) return ORC_E_MEM;
  memcpy(U, F, sizeof(double) * n);
  for (int t = 0; t < p->iters && rc == ORC_OK; ++t) {
    if (saved) memcpy(saved + (size_t)(2 * t) * n, U, sizeof(double) * n);
    rc = orc_col_pass(C, M, N, U, g, tmp, p, NULL);
    if (rc) break;
    if (saved) memcpy(saved + (size_t)(2 * t + 1) * n, tmp, sizeof(double) * n);
    rc = orc_row_pass(C, M, N, tmp, g, U, p, NULL);
  }
  free(tmp);
  return rc;
}

/* Adjoint of one column pass.  Given the pass input X, the guidance g and the
 * gradient Yb of a scalar loss with respect to the pass output, writes the
 * gradient with respect to X into Xb, ADDS the gradient with respect to g into
 * gb (M x N) and ADDS the gradient with respect to lambda into *lb.
 * For every subsystem: v = (Yb / cnt)[pixels], ubar = A^{-1} v,
 * u = A^{-1} X[pixels] (recomputed), and for every edge (p, q = p+d) the term
 * t = -sum_c (ubar_p - ubar_q)(u_p - u_q) gives dloss/dw = lambda*t and
 * dloss/dlambda = sum w*t. */
int orc_col_pass_backward(int C, int M, int N, const double* X, const double* g,
                          const double* Yb, double* Xb, double* gb, double* lb,
                          const orc_params* p) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (C < 1 || !X || !g || !Yb || !Xb || !gb || !lb) return ORC_E_ARG;
  int r = p->r, s = (2 * r + 1) * M;
  int nK = orc_centres(N, r, p->stride, NULL);
  int* K = (int*)malloc(sizeof(int) * nK);
  double* cn = (double*)calloc((size_t)M * N, sizeof(double));
  double* Ub = (double*)malloc(sizeof(double) * (size_t)nK * s * C);   /* ubar per strip */
  double* Gb = (double*)malloc(sizeof(double) * (size_t)nK * s);       /* dloss/dg per element */
  double* Lk = (double*)malloc(sizeof(double) * (size_t)nK);           /* dloss/dlambda per strip */
  if (!K || !cn || !Ub || !Gb || !Lk) { free(K); free(cn); free(Ub); free(Gb); free(Lk); return ORC_E_MEM; }
  orc_centres(N, r, p->stride, K);
  for (int ki = 0; ki < nK; ++ki)
    for (int q = 0; q < s; ++q) {
      int i, j;
      orc_snake_pixel(K[ki], r, q, &i, &j);
      cn[(size_t)i * N + j] += 1.0;
    }
  int err = 0;
#pragma omp parallel
  {
    double* diag = (double*)malloc(sizeof(double) * s);
    double* off = (double*)malloc(sizeof(double) * (size_t)s * r);
    double* w = (double*)malloc(sizeof(double) * (size_t)s * r);
    double* Lb = (double*)malloc(sizeof(double) * (size_t)s * r);
    double* D = (double*)malloc(sizeof(double) * s);
    double* rhs = (double*)malloc(sizeof(double) * (size_t)s * 2 * C);
#pragma omp for schedule(static)
    for (int ki = 0; ki < nK; ++ki) {
      int k = K[ki];
      orc_strip_band(M, N, g, p, k, diag, off, w);
      for (int q = 0; q < s; ++q) {
        int i, j;
        orc_snake_pixel(k, r, q, &i, &j);
        for (int c = 0; c < C; ++c) {
          rhs[(size_t)q * 2 * C + c] = X[((size_t)c * M + i) * N + j];
          rhs[(size_t)q * 2 * C + C + c] = Yb[((size_t)c * M + i) * N + j] / cn[(size_t)i * N + j];
        }
      }
      if (band_ldlt_solve_ws(s, r, diag, off, 2 * C, rhs, Lb, D) != ORC_OK) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      double* ub = Ub + (size_t)ki * s * C;
      double* gk = Gb + (size_t)ki * s;
      for (int q = 0; q < s; ++q) {
        for (int c = 0; c < C; ++c) ub[(size_t)q * C + c] = rhs[(size_t)q * 2 * C + C + c];
        gk[q] = 0.0;
      }
      double lsum = 0.0;
      for (int q = 0; q < s; ++q) {
        int iq, jq;
        orc_snake_pixel(k, r, q, &iq, &jq);
        for (int d = 1; d <= r && q + d < s; ++d) {
          int ie, je;
          orc_snake_pixel(k, r, q + d, &ie, &je);
          double t = 0.0;
          for (int c = 0; c < C; ++c) {
            double du = rhs[(size_t)q * 2 * C + c] - rhs[(size_t)(q + d) * 2 * C + c];
            double dub = rhs[(size_t)q * 2 * C + C + c] - rhs[(size_t)(q + d) * 2 * C + C + c];
            t -= dub * du;
          }
          lsum += w[(size_t)q * r + d - 1] * t;
          double wbar = p->lambda * t;
          double dw = orc_weight_dga(p, d, g[(size_t)iq * N + jq], g[(size_t)ie * N + je]);
          gk[q] += wbar * dw;
          gk[q + d] -= wbar * dw;
        }
      }
      Lk[ki] = lsum;
    }
    free(diag); free(off); free(w); free(Lb); free(D); free(rhs);
  }
  if (!err) {
    memset(Xb, 0, sizeof(double) * (size_t)C * M * N);
    for (int ki = 0; ki < nK; ++ki) {
      const double* ub = Ub + (size_t)ki * s * C;
      const double* gk = Gb + (size_t)ki * s;
      for (int q = 0; q < s; ++q) {
        int i, j;
        orc_snake_pixel(K[ki], r, q, &i, &j);
        for (int c = 0; c < C; ++c) Xb[((size_t)c * M + i) * N + j] += ub[(size_t)q * C + c];
        gb[(size_t)i * N + j] += gk[q];
      }
      *lb += Lk[ki];
    }
  }
  free(K); free(cn); free(Ub); free(Gb); free(Lk);
  return err ? ORC_E_PIVOT : ORC_OK;
}

/* Adjoint of one row pass (the column pass of the transposed image). */
int orc_row_pass_backward(int C, int M, int N, const double* X, const double* g,
                          const double* Yb, double* Xb, double* gb, double* lb,
                          const orc_params* p) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (C < 1 || !X || !g || !Yb || !Xb || !gb || !lb) return ORC_E_ARG;
  size_t n = (size_t)C * M * N;
  double* Xt = (double*)calloc(n, sizeof(double));
  double* Ybt = (double*)calloc(n, sizeof(double));
  double* Xbt = (double*)calloc(n, sizeof(double));
  double* gt = (double*)calloc((size_t)M * N, sizeof(double));
  double* gbt = (double*)calloc((size_t)M * N, sizeof(double));
  if (!Xt || !Ybt || !Xbt || !gt || !gbt) { free(Xt); free(Ybt); free(Xbt); free(gt); free(gbt); return ORC_E_MEM; }
  transpose_planes(C, M, N, X, Xt);
  transpose_planes(C, M, N, Yb, Ybt);
  transpose_planes(1, M, N, g, gt);
  rc = orc_col_pass_backward(C, N, M, Xt, gt, Ybt, Xbt, gbt, lb, p);
  if (rc == ORC_OK) {
    transpose_planes(C, N, M, Xbt, Xb);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < N; ++j) gb[(size_t)i * N + j] += gbt[(size_t)j * M + i];
  }
  free(Xt); free(Ybt); free(Xbt); free(gt); free(gbt);
  return rc;
}

/* Adjoint of the whole filter.  saved holds the 2T pass inputs written by
 * orc_filter; Ub is the gradient with respect to the filter output.  Writes
 * Fb (gradient w.r.t. F), gb (w.r.t. g) and *lb (w.r.t. lambda). */
int orc_filter_backward(int C, int M, int N, const double* g, const double* saved,
                        const double* Ub, double* Fb, double* gb, double* lb,
                        const orc_params* p) {
  int rc = check_params(p, M, N);
  if (rc) return rc;
  if (p->iters < 1 || C < 1) return ORC_E_ARG;
  size_t n = (size_t)C * M * N;
  double* ybar = (double*)malloc(sizeof(double) * n);
  double* xbar = (double*)malloc(sizeof(double) * n);
  if (!ybar || !xbar) { free(ybar); free(xbar); return ORC_E_MEM; }
  memcpy(ybar, Ub, sizeof(double) * n);
  memset(gb, 0, sizeof(double) * (size_t)M * N);
  *lb = 0.0;
  for (int ps = 2 * p->iters - 1; ps >= 0 && rc == ORC_OK; --ps) {
    const double* X = saved + (size_t)ps * n;
    if (ps % 2 == 0)
      rc = orc_col_pass_backward(C, M, N, X, g, ybar, xbar, gb, lb, p);
    else
      rc = orc_row_pass_backward(C, M, N, X, g, ybar, xbar, gb, lb, p);
    double* t = ybar; ybar = xbar; xbar = t;
  }
  if (rc == ORC_OK) memcpy(Fb, ybar, sizeof(double) * n);
  free(ybar); free(xbar);
  return rc;
}
