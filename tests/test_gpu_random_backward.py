"""Gradients (f, g and lambda) against the FP64 oracle's adjoint over
randomly drawn valid parameters (fixed seed): shapes from one window up to 96
pixels a side, r = 1..4, every stride 1..2r+1, 1-4 channels, T = 1..2, both
weight kinds (alpha_r in [1, 1.5] for omega^frac), the default (automatic)
precision and FP64 pivots.

Every gradient must be finite, and all three are held to 1e-4 normwise.  The
automatic precision takes FP64 pivots for a forward that saves its pass
inputs and for a backward that asks for the lambda gradient: that gradient is
a sum over all edges of terms of both signs, each the product of two
neighbour differences of the solutions, and with a random output gradient it
cancels to a small fraction of its terms (float32 pivots reached 6e-4 here,
also at kappa = 2.5).  A separate test holds the float32 f and g gradients
where they are well conditioned.

Also a regression test: the guidance gradient with omega^frac and
alpha_r > 38.5 / 30 was NaN, because |dG|^alpha_r overflowed float32 for the
sentinel guidance of rows outside the image and the derivative formed
inf * 0."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-4
N_CASES = 80


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_random_parameters_gradients_match_oracle(ops):
    rng = np.random.default_rng(20261203)
    worst = {}
    bad = []
    for i in range(N_CASES):
        r = int(rng.integers(1, 5))
        M, N = int(rng.integers(2 * r + 1, 96)), int(rng.integers(2 * r + 1, 96))
        C, T = int(rng.integers(1, 5)), int(rng.integers(1, 3))
        stride = int(rng.integers(1, 2 * r + 2))
        kind = "exp" if rng.uniform() < 0.7 else "frac"
        lam = float(2.0 ** rng.uniform(-3, 4 if kind == "exp" else 1))
        prec = "fp64_pivot" if rng.uniform() < 0.4 else "auto"
        pd = dict(lam=lam, r=r, iters=T, stride=stride, kind=kind, sigma_s=float(r),
                  sigma_r=float(rng.uniform(0.1, 0.5)), alpha_s=1.2,
                  alpha_r=float(rng.uniform(1.0, 1.5)), eps=1e-4)
        f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
        g = rng.uniform(0, 1, (M, N)).astype(np.float32)
        ubar = rng.standard_normal((C, M, N)).astype(np.float32)
        print(f"[random-bwd] {i} {f.shape} {pd} {prec}", flush=True)
        p = ops.Params(**pd, prec=prec)
        fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
        saved = torch.empty((2 * T, C, M, N), dtype=torch.float32, device="cuda")
        ops.sgwls_filter(fd, gd, p, saved=saved)
        gf, gg, gl = ops.sgwls_backward(gd, saved, torch.from_numpy(ubar).cuda(), p)
        torch.cuda.synchronize()
        P = oracle.OracleParams(**pd)
        _, ref_saved = oracle.filter(f.astype(np.float64), g.astype(np.float64), P, save=True)
        rf, rg, rl = oracle.filter_backward(g.astype(np.float64), ref_saved,
                                            ubar.astype(np.float64), P)
        errs = (rel(gf.cpu().numpy(), rf), rel(gg.cpu().numpy(), rg), rel(gl.item(), rl))
        print(f"[random-bwd] {i} errors f {errs[0]:.2e} g {errs[1]:.2e} lambda {errs[2]:.2e}"
              f" (nan: gpu {bool(np.isnan(gg.cpu().numpy()).any())} oracle {bool(np.isnan(rg).any())})",
              flush=True)
        key = f"{prec}/{kind}"
        worst[key] = max(worst.get(key, 0.0), max(errs))
        if not all(np.isfinite(errs)) or any(e > TOL for e in errs):
            bad.append((i, prec, pd, errs))
    print("[random-bwd] worst", {k: f"{v:.2e}" for k, v in sorted(worst.items())}, flush=True)
    assert not bad, bad


def test_float32_input_and_guidance_gradients(ops):
    """Explicit float32 (no lambda gradient), omega^exp with kappa <= 64: the f
    and g gradients stay within 1e-4 of the oracle's adjoint."""
    rng = np.random.default_rng(20261204)
    for i in range(12):
        r = int(rng.integers(1, 5))
        M, N = int(rng.integers(2 * r + 1, 80)), int(rng.integers(2 * r + 1, 80))
        C, T = int(rng.integers(1, 4)), int(rng.integers(1, 3))
        pd = dict(lam=float(2.0 ** rng.uniform(-3, 2)), r=r, iters=T, stride=int(rng.integers(1, 2 * r + 2)),
                  kind="exp", sigma_s=float(r), sigma_r=float(rng.uniform(0.1, 0.5)), alpha_s=1.2,
                  alpha_r=1.2, eps=1e-4)
        f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
        g = rng.uniform(0, 1, (M, N)).astype(np.float32)
        ubar = rng.standard_normal((C, M, N)).astype(np.float32)
        p = ops.Params(**pd, prec="fp32")
        fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
        saved = torch.empty((2 * T, C, M, N), dtype=torch.float32, device="cuda")
        ops.sgwls_filter(fd, gd, p, saved=saved)
        gf, gg, _ = ops.sgwls_backward(gd, saved, torch.from_numpy(ubar).cuda(), p, want_lambda=False)
        torch.cuda.synchronize()
        P = oracle.OracleParams(**pd)
        _, ref_saved = oracle.filter(f.astype(np.float64), g.astype(np.float64), P, save=True)
        rf, rg, _ = oracle.filter_backward(g.astype(np.float64), ref_saved, ubar.astype(np.float64), P)
        errs = (rel(gf.cpu().numpy(), rf), rel(gg.cpu().numpy(), rg))
        print(f"[fp32-bwd] {i} {pd} errors f {errs[0]:.2e} g {errs[1]:.2e}", flush=True)
        assert max(errs) <= TOL, (i, pd, errs)


@pytest.mark.parametrize("alpha_r", [1.2, 1.3, 1.5, 2.0])
def test_frac_guidance_gradient_is_finite_for_large_alpha(ops, alpha_r):
    rng = np.random.default_rng(77)
    C, M, N = 2, 37, 29
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    ubar = rng.standard_normal((C, M, N)).astype(np.float32)
    pd = dict(lam=0.5, r=2, iters=1, stride=1, kind="frac", sigma_s=2.0, sigma_r=0.2,
              alpha_s=1.2, alpha_r=alpha_r, eps=1e-4)
    p = ops.Params(**pd, prec="fp64_pivot")
    fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    saved = torch.empty((2, C, M, N), dtype=torch.float32, device="cuda")
    ops.sgwls_filter(fd, gd, p, saved=saved)
    gf, gg, gl = ops.sgwls_backward(gd, saved, torch.from_numpy(ubar).cuda(), p)
    torch.cuda.synchronize()
    P = oracle.OracleParams(**pd)
    _, ref_saved = oracle.filter(f.astype(np.float64), g.astype(np.float64), P, save=True)
    rf, rg, rl = oracle.filter_backward(g.astype(np.float64), ref_saved, ubar.astype(np.float64), P)
    gg = gg.cpu().numpy()
    assert np.isfinite(gg).all()
    assert rel(gg, rg) <= TOL and rel(gf.cpu().numpy(), rf) <= TOL and rel(gl.item(), rl) <= TOL
