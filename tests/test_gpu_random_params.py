"""Parity with the FP64 oracle over randomly drawn valid parameters (fixed
seed): shapes from one window up to 160 pixels a side, r = 1..4, every
stride 1..2r+1, 1-5 channels, T = 1..3, lambda log-uniform, both weight kinds
(random alpha_r for omega^frac), and three precision modes: the default
(automatic), FP64 pivots and the float32 excess-pivot mode.  Every draw is held
to 1e-5.

The automatic mode picks float32 when the host bound kappa on lambda * omega
is at most 64 and FP64 pivots above it; with uniform random guidance,
omega^frac reaches about 1/epsilon between near-equal neighbours, so its draws
take FP64 pivots."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5
N_CASES = 150


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def draw(rng):
    r = int(rng.integers(1, 5))
    M, N = int(rng.integers(2 * r + 1, 160)), int(rng.integers(2 * r + 1, 160))
    C, T = int(rng.integers(1, 6)), int(rng.integers(1, 4))
    stride = int(rng.integers(1, 2 * r + 2))
    kind = "exp" if rng.uniform() < 0.7 else "frac"
    lam = float(2.0 ** rng.uniform(-3, 6 if kind == "exp" else 3))
    prec = ["auto", "fp64_pivot", "fp32_delta"][int(rng.integers(0, 3))]
    if prec == "fp32_delta" and r != 1:
        prec = "auto"
    pd = dict(lam=lam, r=r, iters=T, stride=stride, kind=kind, sigma_s=float(r),
              sigma_r=float(rng.uniform(0.05, 0.5)), alpha_s=1.2,
              alpha_r=float(rng.uniform(0.8, 1.5)), eps=1e-4)
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    return f, g, pd, prec


def test_random_parameters_match_oracle(ops):
    rng = np.random.default_rng(20261202)
    worst = {}
    bad = []
    for i in range(N_CASES):
        f, g, pd, prec = draw(rng)
        print(f"[random] {i} {f.shape} {pd} {prec}", flush=True)
        u = ops.sgwls_filter(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(),
                             ops.Params(**pd, prec=prec))
        torch.cuda.synchronize()
        ref = oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))
        e = float(np.abs(u.cpu().numpy().astype(np.float64) - ref).max() / np.abs(ref).max())
        if prec == "auto":
            prec = "auto:" + ops.resolve_precision(ops.Params(**pd, prec="auto"))
        key = f"{prec}/{pd['kind']}"
        worst[key] = max(worst.get(key, 0.0), e)
        if not np.isfinite(e) or e > TOL:
            bad.append((i, prec, pd, e))
    print("[random] worst", {k: f"{v:.2e}" for k, v in sorted(worst.items())}, flush=True)
    assert not bad, bad


@pytest.mark.parametrize("alpha_r", [0.0, 0.1, 0.2])
@pytest.mark.parametrize("prec", ["fp32", "fp64_pivot"])
def test_frac_small_alpha_at_the_border(ops, alpha_r, prec):
    # Regression: rows outside the image carry a padding guidance, and with
    # omega^frac and a small alpha_r the edges to them kept a weight (up to
    # 1 / (1 + eps) at alpha_r = 0), which coupled the border pixels to the
    # padding: 72 % error at the image corner.
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 1, (2, 37, 45)).astype(np.float32)
    g = rng.uniform(0, 1, (37, 45)).astype(np.float32)
    pd = dict(lam=10.0, r=1, iters=1, stride=1, kind="frac", sigma_s=1.0, sigma_r=0.1,
              alpha_s=1.2, alpha_r=alpha_r, eps=1e-4)
    u = ops.sgwls_filter(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(),
                         ops.Params(**pd, prec=prec))
    torch.cuda.synchronize()
    ref = oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))
    e = float(np.abs(u.cpu().numpy().astype(np.float64) - ref).max() / np.abs(ref).max())
    assert e <= TOL, e
