"""Pins for the FP64 CPU oracle: it is checked against things the paper and the
mathematics fix, not against itself.

* the paper's worked neighbourhood example (Sec. 2.1)            -> snake order
* dense LU (numpy) of every assembled subsystem                   -> the band solver
* the paper's own r-band LU, Eqs. (9)-(20), written from the text  -> the band solver
* DCT-II closed form of I + lambda*w*L_path (uniform weights)      -> assembly, solver, scatter, averaging
* 2x2 closed form                                                  -> solver at the smallest size
* a constant image passes unchanged; lambda = 0 is the identity    -> row sums of A_s, averaging
* A_s symmetric, rows sum to one, an M-matrix (inverse >= 0)       -> assembly signs
* max principle min F <= U <= max F                                -> solver sign and stability
* linearity, channel independence, transpose equivariance          -> pass structure
* closed-form subsystem counts per pixel (stride 1 and 2r+1)       -> centres, averaging
* hand-derived weight values, central differences of the weight    -> Eq. (2) and its derivative
* isolated bright guidance pixel: exactly its edges vanish         -> which pixels are paired, at which d
* central finite differences of the whole filter (h = 1e-3)        -> the adjoint
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import OracleParams

RNG = np.random.default_rng(12345)


def dense_from_band(diag, off):
    s, r = off.shape
    A = np.diag(diag.copy())
    for p in range(s):
        for d in range(1, r + 1):
            if p + d < s:
                A[p, p + d] = off[p, d - 1]
                A[p + d, p] = off[p, d - 1]
    return A


# ---------------------------------------------------------------- snake order

def test_snake_matches_paper_example():
    # tests/golden/snake_3x3_r1.txt: Sec. 2.1, 3x3 image labelled 1..9 row-major.
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "snake_3x3_r1.txt")
    with open(path) as fh:
        lines = [ln for ln in fh if not ln.startswith("#") and ln.strip()]
    expected = [int(v) for v in lines[0].split()]
    labels = np.arange(1, 10).reshape(3, 3)
    got = [labels[oracle.snake_pixel(1, 1, p)] for p in range(9)]
    assert got == expected
    pos5 = got.index(5)
    assert {got[pos5 - 1], got[pos5 + 1]} == {4, 6}


def test_snake_visits_every_pixel_of_strip_once_and_neighbours_are_in_window():
    for r in (1, 2, 3):
        M, k = 7, 5
        w = 2 * r + 1
        pix = [oracle.snake_pixel(k, r, p) for p in range(w * M)]
        assert len(set(pix)) == w * M
        assert {j for _, j in pix} == set(range(k - r, k + r + 1))
        # Sec. 2.1: any 2r+1 consecutive vector elements are neighbours in the
        # (2r+1)x(2r+1) window system.
        for p in range(w * M):
            for d in range(1, r + 1):
                if p + d < w * M:
                    (i1, j1), (i2, j2) = pix[p], pix[p + d]
                    assert abs(i1 - i2) <= r and abs(j1 - j2) <= r


def test_centres():
    assert list(oracle.centres(7, 1, 1)) == [1, 2, 3, 4, 5]
    assert list(oracle.centres(9, 1, 3)) == [1, 4, 7]          # tiles exactly
    assert list(oracle.centres(10, 1, 3)) == [1, 4, 7, 8]      # last centre appended
    assert list(oracle.centres(5, 2, 5)) == [2]
    with pytest.raises(ValueError):
        oracle.centres(4, 2, 1)


# ---------------------------------------------------------------- weights, Eq. (2)

def test_weight_hand_values():
    pe = OracleParams(kind="exp", sigma_s=1.0, sigma_r=0.1)
    # exp(-1/2) * exp(0): same guidance, neighbours at distance 1
    assert oracle.weight(pe, 1, 0.3, 0.3) == pytest.approx(0.6065306597126334, rel=1e-15)
    # |dG| = sigma_r: exp(-1/2) * exp(-1/2) = exp(-1)
    assert oracle.weight(pe, 1, 0.5, 0.4) == pytest.approx(0.36787944117144233, rel=1e-12)
    # distance 2, sigma_s = 2: exp(-4/8) = exp(-1/2)
    pe2 = OracleParams(kind="exp", sigma_s=2.0, sigma_r=0.1)
    assert oracle.weight(pe2, 2, 0.0, 0.0) == pytest.approx(0.6065306597126334, rel=1e-15)
    pf = OracleParams(kind="frac", alpha_s=1.2, alpha_r=1.2, eps=1e-4)
    # 1/(1 + 1e-4) * 1/(0 + 1e-4)
    assert oracle.weight(pf, 1, 0.2, 0.2) == pytest.approx(9999.000099990001, rel=1e-13)
    # alpha = 1 makes the powers plain: 1/(2 + 1e-4) * 1/(0.5 + 1e-4)
    pf1 = OracleParams(kind="frac", alpha_s=1.0, alpha_r=1.0, eps=1e-4)
    assert oracle.weight(pf1, 2, 0.5, 0.0) == pytest.approx(1.0 / (2.0001 * 0.5001), rel=1e-13)
    # alpha = 2: 1/(4 + 1e-4) * 1/(0.25 + 1e-4)
    pf2 = OracleParams(kind="frac", alpha_s=2.0, alpha_r=2.0, eps=1e-4)
    assert oracle.weight(pf2, 2, 0.0, -0.5) == pytest.approx(1.0 / (4.0001 * 0.2501), rel=1e-13)


@pytest.mark.parametrize("kind", ["exp", "frac"])
def test_weight_derivative_by_central_differences(kind):
    p = OracleParams(kind=kind, sigma_s=1.5, sigma_r=0.2, alpha_s=1.2, alpha_r=1.2)
    for ga, gb in [(0.3, 0.1), (0.1, 0.35), (0.7, 0.69), (-0.2, 0.4)]:
        for d in (1, 2, 3):
            h = 1e-6
            fd = (oracle.weight(p, d, ga + h, gb) - oracle.weight(p, d, ga - h, gb)) / (2 * h)
            assert oracle.weight_dga(p, d, ga, gb) == pytest.approx(fd, rel=1e-5, abs=1e-9)
    assert oracle.weight_dga(OracleParams(kind="frac"), 1, 0.5, 0.5) == 0.0


# ---------------------------------------------------------------- assembly, Eqs. (4)-(5)

@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["exp", "frac"])
def test_assembled_subsystem_is_symmetric_unit_row_sum_m_matrix(r, kind):
    M, N = 6, 2 * r + 3
    g = RNG.uniform(0, 1, (M, N))
    p = OracleParams(lam=3.0, r=r, kind=kind, sigma_s=float(r), sigma_r=0.1)
    diag, off, w = oracle.strip_band(g, p, r + 1)
    A = dense_from_band(diag, off)
    assert np.allclose(A, A.T)
    assert np.allclose(A.sum(axis=1), 1.0, rtol=0, atol=1e-9 * np.abs(A).max())
    assert np.all(np.linalg.eigvalsh(A) > 0)
    off_diag = A - np.diag(np.diag(A))
    assert np.all(off_diag <= 0)
    Ainv = np.linalg.inv(A)
    assert np.all(Ainv >= -1e-12 * np.abs(Ainv).max())          # M-matrix
    assert np.allclose(off, -p.lam * w)


def test_isolated_bright_guidance_pixel_cuts_exactly_its_edges():
    # g = 0 except one pixel; exp range weights with sigma_r = 0.1 give
    # exp(-50) ~ 2e-22 on every edge that touches it and exactly the spatial
    # weight exp(-d^2 / 2 sigma_s^2) everywhere else.
    for r in (1, 2):
        M, N, k = 5, 2 * r + 1, r
        for (bi, bj) in [(2, k), (1, 0), (3, 2 * r)]:
            g = np.zeros((M, N))
            g[bi, bj] = 1.0
            p = OracleParams(lam=1.0, r=r, kind="exp", sigma_s=1.3, sigma_r=0.1)
            _, _, w = oracle.strip_band(g, p, k)
            s = (2 * r + 1) * M
            for q in range(s):
                for d in range(1, r + 1):
                    if q + d >= s:
                        assert w[q, d - 1] == 0.0
                        continue
                    touches = (oracle.snake_pixel(k, r, q) == (bi, bj) or
                               oracle.snake_pixel(k, r, q + d) == (bi, bj))
                    if touches:
                        assert w[q, d - 1] < 1e-20
                    else:
                        # 1D distance d along the vector (reading of Sec. 2.2)
                        assert w[q, d - 1] == pytest.approx(math.exp(-d * d / (2 * 1.3 ** 2)))


# ---------------------------------------------------------------- exact subsystem solve, Eq. (5)

@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["exp", "frac"])
def test_band_solve_matches_dense_lu(r, kind):
    for M in (2 * r + 1, 7):
        N = 2 * r + 4
        g = RNG.uniform(0, 1, (M, N))
        p = OracleParams(lam=float(RNG.uniform(0.5, 30)), r=r, kind=kind, sigma_s=float(r))
        for k in oracle.centres(N, r, 1):
            diag, off, _ = oracle.strip_band(g, p, int(k))
            A = dense_from_band(diag, off)
            f = RNG.normal(size=(len(diag), 3))
            u = oracle.band_solve(diag, off, f)
            ref = np.linalg.solve(A, f)
            assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()
            assert np.linalg.norm(A @ u - f) <= 1e-13 * np.linalg.norm(f) * np.linalg.cond(A)


def r_band_lu_solve(a, b, f, r):
    """The paper's r-band LU, Eqs. (9)-(14), then Eqs. (15)-(17) and (18)-(20),
    1-based as printed and evaluated row by row in k.  A_s is symmetric, so
    c_{k,i} = b_{k,i} = A_s(k, k+i)."""
    s = len(a)
    A = lambda k: a[k - 1]
    B = lambda k, i: b[k - 1][i - 1]
    alpha, gam, beta = {}, {}, {}
    for k in range(1, s + 1):
        if k == 1:                                                  # Eq. (9)
            alpha[1] = A(1)
            for i in range(1, r + 1):
                if 1 + i <= s:
                    gam[1, i] = B(1, i)
                    beta[1, i] = B(1, i) / alpha[1]
            continue
        if k <= r:                                                  # Eq. (10)
            alpha[k] = A(k) - sum(gam[k - t, t] * beta[k - t, t] for t in range(1, k))
            for i in range(1, r - k + 2):
                if k + i <= s:
                    gam[k, i] = B(k, i) - sum(gam[k - t, i + t] * beta[k - t, t] for t in range(1, k))
                    beta[k, i] = (B(k, i) - sum(beta[k - t, i + t] * gam[k - t, t]
                                                for t in range(1, k))) / alpha[k]
            for i in range(r - k + 2, r):                           # Eq. (11), k >= 3
                if k >= 3 and k + i <= s:
                    gam[k, i] = B(k, i) - sum(gam[k - t, i + t] * beta[k - t, t] for t in range(1, r - i + 1))
                    beta[k, i] = (B(k, i) - sum(beta[k - t, i + t] * gam[k - t, t]
                                                for t in range(1, r - i + 1))) / alpha[k]
        else:                                                       # Eq. (12)
            alpha[k] = A(k) - sum(gam[k - t, t] * beta[k - t, t] for t in range(1, r + 1))
            if k <= s - 1:                                          # Eq. (13)
                for i in range(1, min(r - 1, s - k) + 1):
                    gam[k, i] = B(k, i) - sum(gam[k - t, i + t] * beta[k - t, t] for t in range(1, r - i + 1))
                    beta[k, i] = (B(k, i) - sum(beta[k - t, i + t] * gam[k - t, t]
                                                for t in range(1, r - i + 1))) / alpha[k]
        if 2 <= k <= s - r:                                         # Eq. (14)
            gam[k, r] = B(k, r)
            beta[k, r] = B(k, r) / alpha[k]
    y = {}
    y[1] = f[0] / alpha[1]                                          # Eq. (15)
    for k in range(2, s + 1):
        if k <= r:                                                  # Eq. (16)
            y[k] = (f[k - 1] - sum(gam[t, k - t] * y[t] for t in range(1, k))) / alpha[k]
        else:                                                       # Eq. (17)
            y[k] = (f[k - 1] - sum(gam[k - t, t] * y[k - t] for t in range(1, r + 1))) / alpha[k]
    u = {s: y[s]}                                                   # Eq. (18)
    for k in range(s - 1, 0, -1):
        if k >= s - r + 1:                                          # Eq. (19)
            u[k] = y[k] - sum(beta[k, t] * u[k + t] for t in range(1, s - k + 1))
        else:                                                       # Eq. (20)
            u[k] = y[k] - sum(beta[k, t] * u[k + t] for t in range(1, r + 1))
    return np.array([u[k] for k in range(1, s + 1)])


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_band_solve_matches_paper_r_band_lu(r):
    for M in (2 * r + 1, 5):
        N = 2 * r + 2
        g = RNG.uniform(0, 1, (M, N))
        p = OracleParams(lam=7.0, r=r, kind="exp", sigma_s=float(r), sigma_r=0.2)
        diag, off, _ = oracle.strip_band(g, p, r)
        f = RNG.normal(size=len(diag))
        u_lu = r_band_lu_solve(diag, off, f, r)
        u = oracle.band_solve(diag, off, f)
        assert np.abs(u - u_lu).max() <= 1e-12 * np.abs(u).max()


def test_two_by_two_closed_form():
    # [[1+a, -a], [-a, 1+a]] u = f  ->  u1 = ((1+a) f1 + a f2) / (1+2a)
    for a in (0.0, 0.3, 5.0, 1e4):
        f = np.array([0.7, -1.9])
        u = oracle.band_solve(np.array([1 + a, 1 + a]), np.array([[-a], [0.0]]), f)
        assert u[0] == pytest.approx(((1 + a) * f[0] + a * f[1]) / (1 + 2 * a), rel=1e-13)
        assert u[1] == pytest.approx(((1 + a) * f[1] + a * f[0]) / (1 + 2 * a), rel=1e-13)


def dct_path_solve(f, lw):
    """u = (I + lw * L_path)^{-1} f through the DCT-II eigenbasis of the path
    Laplacian: eigenvalues 2 - 2 cos(pi k / s)."""
    s = len(f)
    eig = 2.0 - 2.0 * np.cos(np.pi * np.arange(s) / s)
    return scipy.fft.idct(scipy.fft.dct(f, type=2, norm="ortho") / (1.0 + lw * eig),
                          type=2, norm="ortho")


def test_uniform_weights_strip_solve_matches_dct_closed_form():
    M, N, r = 9, 6, 1
    g = np.full((M, N), 0.37)
    for lam in (0.5, 4.0, 900.0):
        p = OracleParams(lam=lam, r=r, kind="exp", sigma_s=1.0, sigma_r=0.1)
        diag, off, _ = oracle.strip_band(g, p, 2)
        f = RNG.normal(size=len(diag))
        u = oracle.band_solve(diag, off, f)
        ref = dct_path_solve(f, lam * math.exp(-0.5))
        assert np.abs(u - ref).max() <= 1e-12 * max(1.0, lam) * np.abs(ref).max()


def paper_strip_vector_indices(M, k, r):
    """Sec. 2.1 as written, 1-based rows: take columns k-r..k+r, reverse the
    row vectors of even rows, concatenate head to end.  Returns (row, col)
    0-based pairs in vector order."""
    out = []
    for i1 in range(1, M + 1):
        row = [(i1 - 1, j) for j in range(k - r, k + r + 1)]
        if i1 % 2 == 0:
            row = row[::-1]
        out.extend(row)
    return out


@pytest.mark.parametrize("stride", [1, 2, 3])
def test_uniform_guidance_pass_matches_dct_pass(stride):
    # Whole column pass with constant guidance, built independently: Sec. 2.1
    # construction, DCT closed-form solve, inverse construction, averaging.
    M, N, C, r, lam = 8, 11, 2, 1, 3.0
    g = np.full((M, N), -0.2)
    X = RNG.normal(size=(C, M, N))
    p = OracleParams(lam=lam, r=r, stride=stride, kind="exp", sigma_s=1.0)
    Y, cnt = oracle.col_pass(X, g, p)
    ks = list(range(r, N - r, stride))
    if ks[-1] != N - 1 - r:
        ks.append(N - 1 - r)
    acc = np.zeros_like(X)
    cn = np.zeros((M, N))
    for k in ks:
        idx = paper_strip_vector_indices(M, k, r)
        for c in range(C):
            f = np.array([X[c, i, j] for i, j in idx])
            u = dct_path_solve(f, lam * math.exp(-0.5))
            for (i, j), v in zip(idx, u):
                acc[c, i, j] += v
        for i, j in idx:
            cn[i, j] += 1
    assert np.array_equal(cn, cnt)
    assert np.abs(Y - acc / cn).max() <= 1e-12


# ---------------------------------------------------------------- invariants of a pass and of the filter

def random_case(M=9, N=10, C=3, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (C, M, N)), rng.uniform(0, 1, (M, N))


@pytest.mark.parametrize("r,stride", [(1, 1), (2, 1), (2, 3), (3, 7), (1, 3)])
@pytest.mark.parametrize("kind", ["exp", "frac"])
def test_constant_image_passes_unchanged(r, stride, kind):
    X, g = random_case(M=2 * r + 5, N=2 * r + 6)
    X[:] = np.array([0.25, -1.5, 3.0])[:, None, None]
    p = OracleParams(lam=50.0, r=r, iters=2, stride=stride, kind=kind, sigma_s=float(r))
    U = oracle.filter(X, g, p)
    assert np.abs(U - X).max() <= 1e-11


def test_lambda_zero_is_identity():
    X, g = random_case()
    for r in (1, 2):
        U = oracle.filter(X, g, OracleParams(lam=0.0, r=r, iters=2))
        assert np.abs(U - X).max() <= 1e-15


@pytest.mark.parametrize("r", [1, 2, 3])
def test_max_principle(r):
    X, g = random_case(M=10, N=12, seed=r)
    for lam in (0.5, 20.0, 900.0):
        for kind in ("exp", "frac"):
            U = oracle.filter(X, g, OracleParams(lam=lam, r=r, iters=2, kind=kind, sigma_s=float(r)))
            lo = X.min(axis=(1, 2))[:, None, None]
            hi = X.max(axis=(1, 2))[:, None, None]
            assert np.all(U >= lo - 1e-12) and np.all(U <= hi + 1e-12)


def test_linearity_and_channel_independence():
    X1, g = random_case(seed=1)
    X2, _ = random_case(seed=2)
    p = OracleParams(lam=6.0, r=2, iters=2, sigma_s=2.0)
    U = oracle.filter(2.0 * X1 - 0.5 * X2, g, p)
    assert np.abs(U - (2.0 * oracle.filter(X1, g, p) - 0.5 * oracle.filter(X2, g, p))).max() <= 1e-13
    for c in range(3):
        assert np.abs(U[c] - oracle.filter((2.0 * X1 - 0.5 * X2)[c], g, p)).max() <= 1e-13


@pytest.mark.parametrize("r,stride", [(1, 1), (2, 2), (3, 1)])
def test_row_pass_is_transposed_column_pass(r, stride):
    X, g = random_case(M=11, N=9)
    p = OracleParams(lam=5.0, r=r, stride=stride, sigma_s=float(r))
    Yr, cr = oracle.row_pass(X, g, p)
    Yc, cc = oracle.col_pass(X.transpose(0, 2, 1), g.T, p)
    assert np.abs(Yr - Yc.transpose(0, 2, 1)).max() <= 1e-14
    assert np.array_equal(cr, cc.T)


def test_filter_is_alternating_column_then_row_passes():
    X, g = random_case()
    p = OracleParams(lam=3.0, r=1, iters=2)
    Y = X
    for _ in range(2):
        Y, _ = oracle.col_pass(Y, g, p)
        Y, _ = oracle.row_pass(Y, g, p)
    assert np.abs(oracle.filter(X, g, p) - Y).max() <= 1e-15


@pytest.mark.parametrize("r", [1, 2, 3])
def test_subsystem_count_closed_form(r):
    M, N = 2 * r + 3, 5 * (2 * r + 1)
    X, g = random_case(M=M, N=N)
    _, cnt = oracle.col_pass(X, g, OracleParams(r=r, stride=1))
    j = np.arange(N)
    closed = np.minimum(N - 1 - r, j + r) - np.maximum(r, j - r) + 1
    assert np.array_equal(cnt, np.broadcast_to(closed, (M, N)))
    # stride 2r+1 with N a multiple of 2r+1: the strips tile the image
    _, cnt = oracle.col_pass(X, g, OracleParams(r=r, stride=2 * r + 1))
    assert np.all(cnt == 1)


def test_tiling_stride_gives_the_strip_solutions_untouched():
    r, M, N = 1, 6, 9
    X, g = random_case(M=M, N=N)
    p = OracleParams(lam=4.0, r=r, stride=3)
    Y, _ = oracle.col_pass(X, g, p)
    for k in (1, 4, 7):
        diag, off, _ = oracle.strip_band(g, p, k)
        idx = paper_strip_vector_indices(M, k, r)
        f = np.stack([[X[c, i, j] for i, j in idx] for c in range(3)], axis=1)
        A = dense_from_band(diag, off)
        u = np.linalg.solve(A, f)
        for n, (i, j) in enumerate(idx):
            assert np.abs(Y[:, i, j] - u[n]).max() <= 1e-13


def test_rejects_bad_arguments():
    X, g = random_case()
    for bad in (dict(r=0), dict(stride=4), dict(lam=-1.0), dict(lam=float("nan")),
                dict(sigma_r=0.0), dict(r=5)):
        with pytest.raises(ValueError):
            oracle.filter(X, g, OracleParams(**bad))


# ---------------------------------------------------------------- sparse interpolation, Eq. (21)

def test_sparse_interpolation_reproduces_constants_and_known_field():
    rng = np.random.default_rng(7)
    M, N = 12, 13
    g = rng.uniform(0, 1, (M, N))
    H = (rng.uniform(size=(M, N)) < 0.2).astype(np.float64)
    p = OracleParams(lam=50.0, r=2, iters=2, stride=2, sigma_s=2.0, sigma_r=3.0)
    U = oracle.sparse_interpolate(0.8 * H, H, g, p)
    assert np.abs(U - 0.8).max() <= 1e-12
    ones = np.ones((M, N))
    F = rng.normal(size=(M, N))
    assert np.abs(oracle.sparse_interpolate(F, ones, g, p) - oracle.filter(F, g, p)).max() <= 1e-12


# ---------------------------------------------------------------- gradients

def _fd_case(kind, r, stride=1):
    rng = np.random.default_rng(99 + r)
    M, N, C = 6, 7, 2
    F = rng.uniform(0, 1, (C, M, N))
    g = rng.uniform(0, 1, (M, N))
    W = rng.normal(size=(C, M, N))
    p = OracleParams(lam=2.5, r=r, iters=2, stride=stride, kind=kind, sigma_s=float(r),
                     sigma_r=0.3, alpha_s=1.2, alpha_r=1.2)
    return F, g, W, p


@pytest.mark.parametrize("kind,r,stride", [("exp", 1, 1), ("exp", 2, 1), ("exp", 2, 3),
                                           ("frac", 1, 1)])
def test_backward_matches_central_differences(kind, r, stride):
    F, g, W, p = _fd_case(kind, r, stride)
    loss = lambda F_, g_, p_: float(np.sum(W * oracle.filter(F_, g_, p_)))
    U, saved = oracle.filter(F, g, p, save=True)
    Fb, gb, lb = oracle.filter_backward(g, saved, W, p)
    # h = 1e-3 for the smooth exp weight; |dG|^1.2 in omega^frac is sharply
    # curved where two guidance values nearly coincide, so it gets a smaller step.
    h = 1e-3 if kind == "exp" else 1e-5
    fdF = np.zeros_like(F)
    for idx in np.ndindex(F.shape):
        Fp, Fm = F.copy(), F.copy()
        Fp[idx] += h
        Fm[idx] -= h
        fdF[idx] = (loss(Fp, g, p) - loss(Fm, g, p)) / (2 * h)
    assert np.abs(Fb - fdF).max() <= 1e-8 * np.abs(fdF).max()     # linear in F
    fdg = np.zeros_like(g)
    for idx in np.ndindex(g.shape):
        gp_, gm_ = g.copy(), g.copy()
        gp_[idx] += h
        gm_[idx] -= h
        fdg[idx] = (loss(F, gp_, p) - loss(F, gm_, p)) / (2 * h)
    assert np.abs(gb - fdg).max() <= 1e-4 * np.abs(fdg).max()
    from dataclasses import replace
    fdl = (loss(F, g, replace(p, lam=p.lam + h)) - loss(F, g, replace(p, lam=p.lam - h))) / (2 * h)
    assert lb == pytest.approx(fdl, rel=1e-5)


def test_backward_dot_product_identity():
    # <S f, v> = <f, S^T v> for the linear map f -> S f at fixed g.
    F, g, W, p = _fd_case("exp", 2)
    U, saved = oracle.filter(F, g, p, save=True)
    Fb, _, _ = oracle.filter_backward(g, saved, W, p)
    assert np.sum(U * W) == pytest.approx(np.sum(F * Fb), rel=1e-12)
