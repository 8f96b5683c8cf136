"""GPU parity: the HIP library against the FP64 CPU oracle, element by element.

Error measure: normwise relative, max|gpu - oracle| / max|oracle| per output
(the mean is printed beside it).  Bar: 1e-5 for the default precision
(automatic: float32 unless the host bound on lambda * omega asks for FP64
pivots) and for FP64 pivots; explicit float32 is reported where its pivots
lose digits.
"""
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


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    scale = np.abs(ref).max()
    d = np.abs(gpu - ref)
    return d.max() / scale, d.mean() / scale


def run_filter(ops, f, g, pd, prec="auto", **kw):
    p = ops.Params(**pd, prec=prec)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    gt = torch.from_numpy(np.ascontiguousarray(g)).cuda()
    u = ops.sgwls_filter(ft, gt, p, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def oracle_filter(f, g, pd):
    return oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))


def pdict(lam=1.0, r=1, iters=1, stride=1, kind="exp", sigma_r=0.1, alpha=1.2):
    return dict(lam=lam, r=r, iters=iters, stride=stride, kind=kind, sigma_s=float(r),
                sigma_r=sigma_r, alpha_s=alpha, alpha_r=alpha, eps=1e-4)


def check(name, gpu, ref, tol=TOL):
    mx, mean = rel_err(gpu, ref)
    print(f"[parity] {name}: max {mx:.3e} mean {mean:.3e}", flush=True)
    assert mx <= tol, f"{name}: {mx:.3e} > {tol:.1e}"


def test_grey256_r1_T1(ops):
    w = synth.grey256()
    check("grey256 r1 T1", run_filter(ops, w.f, w.g, w.params), oracle_filter(w.f, w.g, w.params))


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("r,stride", [(1, 1), (1, 3), (2, 1), (2, 4), (3, 1), (3, 7), (4, 1), (4, 5)])
@pytest.mark.parametrize("C", [1, 3])
def test_single_pass_small(ops, direction, r, stride, C):
    # several chunks and a ragged last chunk in both directions
    rng = np.random.default_rng(100 * r + 10 * stride + C + direction)
    M, N = 37 + 2 * r, 53 + 3 * r
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=5.0, r=r, stride=stride, sigma_r=0.2)
    p = ops.Params(**pd)
    out = ops.sgwls_pass(direction, torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), p)
    torch.cuda.synchronize()
    fn = oracle.col_pass if direction == 0 else oracle.row_pass
    ref = fn(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))[0]
    check(f"pass dir{direction} r{r} s{stride} C{C}", out.cpu().numpy(), ref)


@pytest.mark.parametrize("r,stride", [(1, 2), (1, 3), (2, 3), (2, 5), (3, 4), (3, 7), (4, 4), (4, 9)])
@pytest.mark.parametrize("C", [1, 3])
def test_strided_filter(ops, r, stride, C):
    # the whole filter (both directions as transposed column passes) at a
    # stride > 1: at least two expand blocks across each frame, several chunks
    # along it and ragged ends, in float32 and with FP64 pivots
    rng = np.random.default_rng(7000 + 100 * r + 10 * stride + C)
    ow = 62 * stride - 2 * r
    M, N = ow + 41 + 3 * r, 2 * ow + 17
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=4.0, r=r, iters=2, stride=stride, sigma_r=0.2)
    ref = oracle_filter(f, g, pd)
    check(f"filter r{r} s{stride} C{C}", run_filter(ops, f, g, pd), ref)
    check(f"filter r{r} s{stride} C{C} fp64", run_filter(ops, f, g, pd, "fp64_pivot"), ref)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("r,stride,C", [(1, 2, 3), (1, 3, 3), (1, 3, 1), (2, 3, 3), (2, 5, 1),
                                        (3, 4, 3), (4, 9, 3)])
def test_strided_variants_match_oracle(ops, r, stride, C, variant):
    # the strided forward variants (two chunks per block; half-height chunks
    # four to a block), pinned on both frames of the filter
    rng = np.random.default_rng(7500 + 100 * r + 10 * stride + C + variant)
    ow = 62 * stride - 2 * r
    M, N = ow + 37 + 5 * r, 2 * ow + 19
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=4.0, r=r, iters=2, stride=stride, sigma_r=0.2)
    p = ops.Params(**pd)
    try:
        try:
            ops.tune_pin(0, C, M, N, p, variant)
            ops.tune_pin(0, C, N, M, p, variant)
        except ops.nat.SgwlsError:
            pytest.skip(f"no strided variant {variant} at r={r}")
        print(f"[parity] strided variant {variant} r{r} s{stride} C{C} {M}x{N}", flush=True)
        check(f"strided variant {variant} r{r} s{stride} C{C}", run_filter(ops, f, g, pd),
              oracle_filter(f, g, pd))
    finally:
        ops.tune_clear()


@pytest.mark.parametrize("prec", ["fp32", "fp64_pivot"])
@pytest.mark.parametrize("r", [3, 4])
def test_multiwave_long_run_solver(ops, r, prec):
    # 700 x 300 at r >= 3 (chunks of two rows): the column frame's 294-ish
    # strips with 349 separators each run the long-run solver with four waves
    # per strip in float32 (two with FP64 pivots, whose exchange is twice as
    # large), the row frame's ~694 strips with two waves per strip
    rng = np.random.default_rng(8100 + r)
    M, N = 700, 300
    f = rng.uniform(0, 1, (3, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=6.0, r=r, iters=1, sigma_r=0.2)
    print(f"[parity] multi-wave long-run solver r{r} {prec}", flush=True)
    check(f"multi-wave long r{r} {prec}", run_filter(ops, f, g, pd, prec), oracle_filter(f, g, pd))


@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("C", [1, 3])
def test_long_lines_use_the_long_run_solver(ops, r, C):
    # lines of 9,000 and 5,000 pixels: more separator blocks per lane than the
    # register interface solver holds, so the scratch-backed solver runs in
    # both directions (tall and wide images)
    for M, N in ((9000, 37), (41, 5000)):
        rng = np.random.default_rng(M + N + 10 * r + C)
        f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
        g = rng.uniform(0, 1, (M, N)).astype(np.float32)
        pd = pdict(lam=5.0, r=r, iters=1, sigma_r=0.2)
        check(f"long lines {M}x{N} r{r} C{C}", run_filter(ops, f, g, pd), oracle_filter(f, g, pd))


@pytest.mark.parametrize("r,M,N", [(1, 65536, 5), (1, 5, 65536), (2, 65536, 7)])
def test_maximum_side(ops, r, M, N):
    # the longest lines the library accepts (65536 pixels): the column or row
    # subsystems have (2r+1) * 65536 elements, solved by the long-run solver
    rng = np.random.default_rng(M + 7 * N + r)
    f = rng.uniform(0, 1, (1, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=5.0, r=r, iters=1, sigma_r=0.2)
    check(f"maximum side {M}x{N} r{r}", run_filter(ops, f, g, pd), oracle_filter(f, g, pd))


@pytest.mark.parametrize("shape", [(3, 3), (3, 4), (4, 3), (5, 200), (200, 5), (7, 7), (2, 9, 9),
                                   (4, 33, 65), (5, 31, 17), (1, 130, 3)])
@pytest.mark.parametrize("r", [1, 2])
def test_edge_shapes(ops, shape, r):
    if len(shape) == 2:
        C, (M, N) = 1, shape
    else:
        C, M, N = shape
    if min(M, N) < 2 * r + 1:
        pytest.skip("smaller than one window")
    rng = np.random.default_rng(M * 1000 + N + C + r)
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=3.0, r=r, iters=2, sigma_r=0.2)
    check(f"shape {shape} r{r}", run_filter(ops, f, g, pd), oracle_filter(f, g, pd))


@pytest.mark.parametrize("kind,lam", [("exp", 0.5), ("exp", 30.0), ("frac", 1.0), ("frac", 5.0)])
@pytest.mark.parametrize("prec", ["auto", "fp32", "fp64_pivot"])
def test_kinds_and_precisions(ops, kind, lam, prec):
    f = synth.image(96, 80, 3, 30, 0.05, seed=11)
    g = synth.luma(f)
    pd = pdict(lam=lam, r=2, iters=2, kind=kind, sigma_r=0.1, alpha=1.2)
    gpu, ref = run_filter(ops, f, g, pd, prec=prec), oracle_filter(f, g, pd)
    if prec == "fp32" and kind == "frac":
        # omega^frac reaches 1/eps = 1e4 where the guidance is flat: lambda*w is
        # large and float32 pivots lose digits to cancellation.  Reported, with
        # a sanity bound; the FP64-pivot mode is the one held to 1e-5.
        mx, mean = rel_err(gpu, ref)
        print(f"[parity] {kind} lam{lam} fp32: max {mx:.3e} mean {mean:.3e}", flush=True)
        assert mx <= 1e-3
    else:
        check(f"{kind} lam{lam} {prec}", gpu, ref)


def test_rgb768x1024_r1_T3(ops):
    w = synth.rgb768x1024()
    check("rgb768x1024 r1 T3", run_filter(ops, w.f, w.g, w.params), oracle_filter(w.f, w.g, w.params))


def test_rgb1080p_r1_T3_bench_config(ops):
    # the configuration bench.py times (1080p RGB, r=1, T=3, lambda=4, stride 1)
    w = synth.rgb1080p()
    check("rgb1080p r1 T3", run_filter(ops, w.f, w.g, w.params), oracle_filter(w.f, w.g, w.params))


@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("lam", [1.0, 16.0, 64.0])
def test_rgb1080p_large_radius_fp64_pivot(ops, r, lam):
    w = synth.rgb1080p(r=r, lam=lam, seed=1002)
    ref = oracle_filter(w.f, w.g, w.params)
    check(f"rgb1080p r{r} lam{lam} fp64_pivot", run_filter(ops, w.f, w.g, w.params, "fp64_pivot"), ref)
    picked = ops.resolve_precision(ops.Params(**w.params, prec="auto"))
    check(f"rgb1080p r{r} lam{lam} auto ({picked})", run_filter(ops, w.f, w.g, w.params), ref)
    # explicit float32: reported (its pivots lose about kappa ulps), sanity bound
    mx, mean = rel_err(run_filter(ops, w.f, w.g, w.params, "fp32"), ref)
    print(f"[parity] rgb1080p r{r} lam{lam} fp32: max {mx:.3e} mean {mean:.3e}", flush=True)
    assert mx <= 1e-4


def test_invariants_on_gpu(ops):
    rng = np.random.default_rng(3)
    M, N = 70, 90
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    const = np.full((3, M, N), 0.625, dtype=np.float32)
    u = run_filter(ops, const, g, pdict(lam=20.0, r=2, iters=2))
    assert np.abs(u - 0.625).max() <= TOL * 0.625     # the same normwise bar
    f = rng.uniform(0, 1, (2, M, N)).astype(np.float32)
    u0 = run_filter(ops, f, g, pdict(lam=0.0, r=1, iters=2))
    assert np.abs(u0 - f).max() <= 4 * np.finfo(np.float32).eps * np.abs(f).max()   # averaging rounds


def test_deterministic_and_in_place(ops):
    w = synth.single("t", 200, 300, 3, 40, 0.05, 5, 4.0, 1, 2)
    a = run_filter(ops, w.f, w.g, w.params)
    b = run_filter(ops, w.f, w.g, w.params)
    assert np.array_equal(a, b)
    ft = torch.from_numpy(w.f.copy()).cuda()
    gt = torch.from_numpy(w.g).cuda()
    p = ops.Params(**w.params)
    ops.sgwls_filter(ft, gt, p, out=ft)
    torch.cuda.synchronize()
    assert np.array_equal(ft.cpu().numpy(), a)


def test_lambda_on_device_and_saved_inputs(ops):
    w = synth.single("t", 64, 96, 3, 20, 0.05, 9, 6.0, 1, 2)
    p = ops.Params(**{**w.params, "lam": 123.0})        # overridden by lambda_dev
    ft = torch.from_numpy(w.f).cuda()
    gt = torch.from_numpy(w.g).cuda()
    lam = torch.tensor([6.0], device="cuda")
    saved = torch.empty(2 * p.iters * w.f.size, device="cuda")
    u = ops.sgwls_filter(ft, gt, p, lambda_dev=lam, saved=saved)
    torch.cuda.synchronize()
    ref, ref_saved = oracle.filter(w.f.astype(np.float64), w.g.astype(np.float64),
                                   oracle.OracleParams(**w.params), save=True)
    check("lambda_dev", u.cpu().numpy(), ref)
    got = saved.cpu().numpy().reshape(ref_saved.shape).copy()
    # stride 1: the row-pass inputs (odd entries) are stored transposed
    C, M, N = w.f.shape
    for q in range(1, got.shape[0], 2):
        got[q] = got[q].reshape(C, N, M).transpose(0, 2, 1)
    check("saved pass inputs", got, ref_saved)


@pytest.mark.parametrize("r,C", [(1, 3), (1, 1), (2, 3), (2, 1)])
@pytest.mark.parametrize("direction", [0, 1])
def test_every_kernel_variant_matches_oracle(ops, r, C, direction):
    rng = np.random.default_rng(10 * r + C + direction)
    M, N = 133, 157                       # several chunks of every variant, ragged
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=6.0, r=r, sigma_r=0.2)
    p = ops.Params(**pd)
    ref = (oracle.col_pass if direction == 0 else oracle.row_pass)(
        f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))[0]
    ft, gt = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    try:
        for v in range(ops.variant_count(r, C)):
            ops.tune_pin(direction, C, M, N, p, v)
            out = ops.sgwls_pass(direction, ft, gt, p)
            torch.cuda.synchronize()
            check(f"variant {v} r{r} C{C} dir{direction}", out.cpu().numpy(), ref)
    finally:
        ops.tune_clear()


@pytest.mark.parametrize("r,C", [(1, 3), (1, 1), (2, 3)])
def test_filter_with_every_pinned_variant_matches_oracle(ops, r, C):
    # The filter with each kernel variant pinned for both frames: pass 0's
    # re-solve also stores the guidance transposed for the row passes (or,
    # for a tile too large for the extra plane, a transpose kernel does).
    rng = np.random.default_rng(100 + 10 * r + C)
    M, N = 133, 157
    f = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    pd = pdict(lam=6.0, r=r, sigma_r=0.2, iters=2)
    p = ops.Params(**pd, prec="fp32")
    ref = oracle.filter(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**pd))
    ft, gt = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    try:
        for v in range(ops.variant_count(r, C)):
            ops.tune_pin(0, C, M, N, p, v)
            ops.tune_pin(0, C, N, M, p, v)
            print(f"[parity] filter, variant {v} pinned, r{r} C{C}", flush=True)
            out = ops.sgwls_filter(ft, gt, p)
            torch.cuda.synchronize()
            check(f"filter variant {v} r{r} C{C}", out.cpu().numpy(), ref)
    finally:
        ops.tune_clear()


def test_autotune_picks_a_variant_and_keeps_parity(ops):
    w = synth.single("t", 300, 420, 3, 40, 0.05, 21, 4.0, 1, 2)
    p = ops.Params(**w.params)
    ft, gt = torch.from_numpy(w.f).cuda(), torch.from_numpy(w.g).cuda()
    try:
        chosen = ops.autotune(ft, gt, p, reps=3)
        assert set(chosen) == {(0, 3), (1, 3)}
        assert ops.tune_query(0, 3, 300, 420, p) == chosen[(0, 3)]
        u = ops.sgwls_filter(ft, gt, p)
        torch.cuda.synchronize()
        check("autotuned filter", u.cpu().numpy(), oracle_filter(w.f, w.g, w.params))
    finally:
        ops.tune_clear()


@pytest.mark.parametrize("prec", ["fp32", "fp64_pivot"])
def test_negative_and_nan_device_lambda(ops, prec):
    """A negative device lambda is clamped to 0 by the kernels (A_s = I + lambda L
    is positive definite only for lambda >= 0), which makes every pass the
    identity; a NaN device lambda propagates to the output."""
    rng = np.random.default_rng(41)
    f = rng.uniform(0, 1, (3, 40, 72)).astype(np.float32)
    g = rng.uniform(0, 1, (40, 72)).astype(np.float32)
    p = ops.Params(**pdict(lam=4.0, r=2, iters=2), prec=prec)
    ft, gt = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    u = ops.sgwls_filter(ft, gt, p, lambda_dev=torch.tensor([-5.0], device="cuda"))
    torch.cuda.synchronize()
    assert np.abs(u.cpu().numpy() - f).max() <= 4 * np.finfo(np.float32).eps
    u = ops.sgwls_filter(ft, gt, p, lambda_dev=torch.tensor([float("nan")], device="cuda"))
    torch.cuda.synchronize()
    assert np.isnan(u.cpu().numpy()).all()
