"""The cancellation-free float32 mode (r = 1): every strip solved serially
by the banded LDL^T of Sec. 2.2 with each pivot carried as its excess over
the coupling still to be eliminated.  Parity with the FP64 oracle at the
float32 bar on ordinary inputs (several strides, channel counts that split
into groups of four, odd shapes, the smallest image, lambda = 0), agreement
with the partitioned float32 path, and the entry points that refuse it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1705_01674_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def params(lam=4.0, iters=2, stride=1, kind="exp"):
    return dict(lam=float(lam), r=1, iters=iters, stride=stride, kind=kind, sigma_s=1.0,
                sigma_r=0.1, alpha_s=1.2, alpha_r=1.2, eps=1e-4)


def gpu(ops, f, g, pd, prec="fp32_delta"):
    p = ops.Params(**pd, prec=prec)
    print(f"[delta] shape {f.shape} {pd} {prec}", flush=True)
    u = ops.sgwls_filter(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), p)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def ref(f, g, pd):
    return oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("M,N,C,stride,iters", [
    (37, 53, 1, 1, 2), (37, 53, 3, 2, 1), (64, 48, 5, 1, 1), (41, 29, 2, 3, 2),
    (96, 128, 3, 1, 3), (3, 3, 1, 1, 1), (3, 17, 4, 3, 2), (130, 7, 1, 2, 1)])
def test_delta_matches_oracle(ops, M, N, C, stride, iters):
    f = synth.image(M, N, C, 20, 0.03, seed=3100 + M + N + C)
    g = synth.luma(f) if C == 3 else f[0].copy()
    pd = params(iters=iters, stride=stride)
    e = rel(gpu(ops, f, g, pd), ref(f, g, pd))
    assert e <= TOL, e


@pytest.mark.parametrize("kind,lam", [("exp", 0.0), ("exp", 1e3), ("frac", 1.0), ("frac", 60.0)])
def test_delta_weights_and_lambda(ops, kind, lam):
    f = synth.image(48, 64, 3, 30, 0.02, seed=3200)
    g = synth.luma(f)
    pd = params(lam=lam, iters=2, kind=kind)
    out = gpu(ops, f, g, pd)
    if lam == 0.0:   # A = I: the identity, up to the rounding of the average
        assert rel(out, f.astype(np.float64)) <= 1e-6
    e = rel(out, ref(f, g, pd))
    assert e <= TOL, e


def test_delta_agrees_with_partitioned_path(ops):
    w = synth.rgb768x1024()
    pd = dict(w.params)
    a = gpu(ops, w.f, w.g, pd)
    b = gpu(ops, w.f, w.g, pd, prec="fp32")
    assert rel(a, b) <= 2 * TOL


def test_delta_in_place_and_lambda_on_device(ops):
    f = synth.image(40, 52, 3, 20, 0.03, seed=3300)
    g = synth.luma(f)
    pd = params(lam=7.0, iters=2)
    want = ref(f, g, pd)
    p = ops.Params(**{**pd, "lam": 1.0}, prec="fp32_delta")
    x = torch.from_numpy(f).cuda()
    lam = torch.tensor([7.0], dtype=torch.float32, device="cuda")
    ops.sgwls_filter(x, torch.from_numpy(g).cuda(), p, lambda_dev=lam, out=x)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy().astype(np.float64), want) <= TOL


def test_delta_refusals(ops):
    from paper_1705_01674_amd import _native as nat
    f = torch.rand(3, 16, 20, device="cuda")
    g = torch.rand(16, 20, device="cuda")
    with pytest.raises(nat.SgwlsError):
        ops.sgwls_filter(f, g, ops.Params(**{**params(), "r": 2}, prec="fp32_delta"))
    saved = torch.empty(4, 3, 16, 20, device="cuda")
    with pytest.raises(nat.SgwlsError):
        ops.sgwls_filter(f, g, ops.Params(**params(), prec="fp32_delta"), saved=saved)


def test_delta_sparse_interpolation(ops):
    # Eq. (21) at r = 1 in this mode (the one filter call over the stacked
    # planes runs serial strips): against the oracle's S(F) / S(H) where the
    # oracle denominator is at least 1e-3.
    w = synth.depth_upsample(72, 96, 4, seed=3400)
    pd = {**w.params, "r": 1, "stride": 1, "sigma_s": 1.0, "lam": 50.0}
    P = oracle.OracleParams(**pd)
    g64 = w.g.astype(np.float64)
    num = oracle.filter(w.f.astype(np.float64), g64, P)
    den = oracle.filter(w.h.astype(np.float64)[None], g64, P)[0]
    mask = den >= 1e-3
    want = num[:, mask] / den[mask]
    p = ops.Params(**pd, prec="fp32_delta")
    print(f"[delta] interpolation {w.f.shape} {pd}", flush=True)
    u = ops.sgwls_interpolate(torch.from_numpy(w.f).cuda(), torch.from_numpy(w.h).cuda(),
                              torch.from_numpy(w.g).cuda(), p)
    torch.cuda.synchronize()
    got = u.cpu().numpy().astype(np.float64)[:, mask]
    assert mask.mean() > 0.9
    assert rel(got, want) <= 1e-4
