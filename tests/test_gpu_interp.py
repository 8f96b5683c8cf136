"""GPU parity of guided sparse interpolation (Eq. 21): sgwls_interpolate
against the FP64 oracle's S(F) / S(H), plus the identities the quotient
satisfies on the GPU itself.

Error measure: normwise relative, max|gpu - oracle| / max|oracle|, over the
pixels whose oracle denominator S(H) is at least 1e-3.  With omega^exp and
the paper's sigma_r = 3 on a 0..255 guidance, an edge whose guidance jump
exceeds about 116 has a weight below the smallest float64 (about 43 in
float32), so a region enclosed by such edges and holding no known sample
gets S(H) = 0 in the oracle or on the GPU, and the quotient 0/0 is undefined
in both; where S(H) is tiny but not 0 the quotient amplifies the rounding of
both filters by 1/S(H).  Those pixels (a fraction of a percent here) are
counted and printed, not compared (at least 90 % of the pixels are).  Bars:
1e-5 for the default (automatic) precision, which takes FP64 pivots for these
r = 4, lambda = 100..900 bands, and for FP64 pivots; with explicit float32
arithmetic the pivots lose accuracy in proportion to lambda (the growth the
dense filter shows at r = 3, lambda = 64), so the float32 bar is 2e-4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1705_01674_amd import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-5
TOL32 = 2e-4


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


DEN_MIN = 1e-3


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    scale = np.abs(ref).max()
    d = np.abs(gpu - ref)
    return d.max() / scale, d.mean() / scale


def run(ops, w, prec="auto", f=None, h=None):
    p = ops.Params(**w.params, prec=prec)
    ft = torch.from_numpy(np.ascontiguousarray(w.f if f is None else f)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(w.h if h is None else h)).cuda()
    gt = torch.from_numpy(np.ascontiguousarray(w.g)).cuda()
    u = ops.sgwls_interpolate(ft, ht, gt, p)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def reference(w):
    """(oracle quotient, mask of the pixels it is compared on)."""
    P = oracle.OracleParams(**w.params)
    g = w.g.astype(np.float64)
    num = oracle.filter(w.f.astype(np.float64), g, P)
    den = oracle.filter(w.h.astype(np.float64), g, P)
    ok = den >= DEN_MIN
    with np.errstate(divide="ignore", invalid="ignore"):
        return num / den, np.broadcast_to(ok, num.shape)


def check(name, gpu, ref_mask, tol):
    ref, ok = ref_mask
    mx, mean = rel_err(gpu[ok], ref[ok])
    print(f"[interp] {name}: max {mx:.3e} mean {mean:.3e} over {ok.mean():.4%} of the pixels",
          flush=True)
    assert np.isfinite(gpu[ok]).all(), name
    assert ok.mean() > 0.9, name
    assert mx <= tol, f"{name}: {mx:.3e} > {tol:.1e}"


@pytest.mark.parametrize("factor", [2, 4, 8])
def test_depth_upsampling_small(ops, factor):
    w = synth.depth_upsample(120, 161, factor=factor, seed=1100 + factor)
    ref = reference(w)
    check(f"depth x{factor} default", run(ops, w), ref, TOL64)
    check(f"depth x{factor} fp64 pivots", run(ops, w, "fp64_pivot"), ref, TOL64)
    check(f"depth x{factor} fp32", run(ops, w, "fp32"), ref, TOL32)


def test_colorization_small(ops):
    w = synth.colorize_scribbles(96, 131, n_strokes=120, seed=1200)
    ref = reference(w)
    check("colorize default", run(ops, w), ref, TOL64)
    check("colorize fp64 pivots", run(ops, w, "fp64_pivot"), ref, TOL64)
    check("colorize fp32", run(ops, w, "fp32"), ref, TOL32)


def test_depth_upsampling_1080p(ops):
    """Full size (1080 x 1920, 8x upsampling, lambda 400) against the whole
    oracle output."""
    w = synth.depth_upsample(1080, 1920, factor=8, seed=1000)
    ref = reference(w)
    check("depth 1080p x8 default", run(ops, w), ref, TOL64)
    check("depth 1080p x8 fp64 pivots", run(ops, w, "fp64_pivot"), ref, TOL64)
    check("depth 1080p x8 fp32", run(ops, w, "fp32"), ref, TOL32)


def test_quotient_identities(ops):
    """F = c H gives c everywhere; H = 1 gives the plain filter of F.  The
    guidance is scaled down so that no weight underflows and S(H) > 0 at
    every pixel."""
    w = synth.depth_upsample(64, 90, factor=4, seed=1300)
    w.g = (0.05 * w.g).astype(np.float32)
    u = run(ops, w, "fp64_pivot", f=(0.8 * w.h)[None].astype(np.float32))
    assert np.abs(u - 0.8).max() <= 1e-5
    ones = np.ones_like(w.h)
    p = ops.Params(**w.params, prec="fp64_pivot")
    ft = torch.from_numpy(w.f).cuda()
    filt = ops.sgwls_filter(ft, torch.from_numpy(w.g).cuda(), p).cpu().numpy()
    u1 = run(ops, w, "fp64_pivot", h=ones)
    assert np.abs(u1 - filt).max() <= 1e-5 * np.abs(filt).max()


def test_interpolation_in_place_and_errors(ops):
    w = synth.depth_upsample(40, 56, factor=2, seed=1400)
    p = ops.Params(**w.params)
    ft = torch.from_numpy(w.f).cuda()
    ht = torch.from_numpy(w.h).cuda()
    gt = torch.from_numpy(w.g).cuda()
    ref = ops.sgwls_interpolate(ft.clone(), ht, gt, p)
    ops.sgwls_interpolate(ft, ht, gt, p, out=ft)          # u aliasing f is allowed
    torch.cuda.synchronize()
    assert torch.equal(ft, ref)
    with pytest.raises(RuntimeError):
        ops.sgwls_interpolate(ft, ht, gt, p, out=gt.view(1, 40, 56))  # u aliasing g
