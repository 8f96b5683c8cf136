"""Precision stress test at the paper's dense-application settings, where
omega^frac (Eq. 2) makes lambda * omega largest: detail enhancement (r = 1,
alpha_s = alpha_r = 1.2, epsilon = 1e-4, lambda = 900) and the three HDR
detail layers (lambda = 5 / 40 / 320 on log luminance).  Float32 pivots
against FP64 pivots and, at r = 1, against the cancellation-free float32
pivots (each pivot carried as its excess over the remaining coupling), all
against the FP64 oracle.

Where the guidance is flat, omega^frac reaches about 1/epsilon = 1e4, so
the pivots are 1 + lambda*sum(omega) with lambda*omega up to 9e6: the 1
that decides the solution along a flat run is about one float32 ulp of the
pivot, and the recurrences cancel the rest.  The default (automatic)
precision, which takes FP64 pivots here, the FP64 pivot mode and the
float32 excess-pivot mode are held to 1e-5 (normwise max, as everywhere);
plain float32 is reported, with only a
finiteness check.  Guidance scales: 0..1 (the
synthetic images), 0..255 (8-bit, as the sparse workloads) and natural-log
luminance for HDR.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1705_01674_amd import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-5


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def frac_params(lam, r=1, iters=3):
    return dict(lam=float(lam), r=r, iters=iters, stride=1, kind="frac", sigma_s=float(r),
                sigma_r=0.1, alpha_s=1.2, alpha_r=1.2, eps=1e-4)


def run(ops, f, g, pd, prec):
    p = ops.Params(**pd, prec=prec)
    u = ops.sgwls_filter(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), p)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def errors(gpu, ref):
    d = np.abs(gpu - ref)
    return d.max() / np.abs(ref).max(), d.mean() / np.abs(ref).max()


def case(ops, name, f, g, pd):
    ref = oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))
    e64, m64 = errors(run(ops, f, g, pd, "fp64_pivot"), ref)
    ea, ma = errors(run(ops, f, g, pd, "auto"), ref)
    u32 = run(ops, f, g, pd, "fp32")
    e32, m32 = errors(u32, ref)
    line = (f"[precision] {name}: fp32 max {e32:.3e} mean {m32:.3e} | fp64 pivots max {e64:.3e} "
            f"mean {m64:.3e} | default max {ea:.3e} mean {ma:.3e}")
    ed = None
    if pd["r"] == 1:   # the cancellation-free float32 pivots exist for r = 1
        ed, md = errors(run(ops, f, g, pd, "fp32_delta"), ref)
        line += f" | fp32 delta pivots max {ed:.3e} mean {md:.3e}"
    print(line, flush=True)
    assert np.isfinite(u32).all(), name
    assert e64 <= TOL64, f"{name}: fp64 pivots {e64:.3e}"
    assert ea <= TOL64, f"{name}: default precision {ea:.3e}"
    if ed is not None:
        assert ed <= TOL64, f"{name}: fp32 delta pivots {ed:.3e}"


@pytest.mark.parametrize("scale", [1.0, 255.0])
@pytest.mark.parametrize("r", [1, 2])
def test_detail_enhancement_lambda900(ops, scale, r):
    img = synth.image(192, 256, 3, 60, 0.02, seed=2100 + r)
    g = (scale * synth.luma(img).astype(np.float64)).astype(np.float32)
    f = (scale * img.astype(np.float64)).astype(np.float32)
    case(ops, f"detail r{r} scale {scale:g} lambda 900", f, g, frac_params(900.0, r))


@pytest.mark.parametrize("lam", [5.0, 40.0, 320.0])
def test_hdr_detail_layers(ops, lam):
    # log luminance of a synthetic HDR image spanning about four decades
    img = synth.image(192, 256, 1, 60, 0.02, seed=2200)[0].astype(np.float64)
    g = np.log(np.exp(9.0 * img) * 1e-2).astype(np.float32)
    f = g[None].copy()
    case(ops, f"hdr log-luminance lambda {lam:g}", f, g, frac_params(lam))
