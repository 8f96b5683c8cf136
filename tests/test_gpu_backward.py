"""GPU parity of the adjoint (backward) kernels against the FP64 CPU oracle.

The oracle's own gradients are pinned to central finite differences and to
the dot-product identity on the CPU (test_oracle_pins.py); here the HIP
backward is compared with them element by element, and a few guidance and
lambda gradients are also checked against central differences of the FP64
oracle directly.  Error measure: normwise relative, max|gpu - ref| / max|ref|.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1705_01674_amd import synth

pytestmark = pytest.mark.gpu

TOL_X = 1e-5      # input gradient: one more solve than the forward pass
TOL_G = 1e-4      # guidance and lambda gradients (products of differences)


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def rel(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(np.abs(ref).max(), 1e-300)
    d = np.abs(gpu - ref)
    return d.max() / scale, d.mean() / scale


def check(name, gpu, ref, tol):
    mx, mean = rel(gpu, ref)
    print(f"[backward] {name}: max {mx:.3e} mean {mean:.3e}", flush=True)
    assert mx <= tol, f"{name}: {mx:.3e} > {tol:.1e}"


def pdict(lam=4.0, r=1, iters=1, stride=1, kind="exp", sigma_r=0.2, alpha=1.2):
    return dict(lam=lam, r=r, iters=iters, stride=stride, kind=kind, sigma_s=float(r),
                sigma_r=sigma_r, alpha_s=alpha, alpha_r=alpha, eps=1e-4)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def inputs(C, M, N, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (M, N)).astype(np.float32)
    yb = rng.standard_normal((C, M, N)).astype(np.float32)
    return x, g, yb


@pytest.mark.parametrize("C", [3, 1])
@pytest.mark.parametrize("r,stride", [(1, 1), (2, 1), (1, 2), (1, 3), (2, 3), (3, 1)])
@pytest.mark.parametrize("direction", [0, 1])
def test_pass_backward_matches_oracle(ops, direction, r, stride, C):
    M, N = 70, 150                        # several chunks and expand blocks, ragged
    x, g, yb = inputs(C, M, N, 100 * r + 10 * stride + C + direction)
    pd = pdict(r=r, stride=stride)
    p = ops.Params(**pd)
    print(f"[backward] pass dir{direction} r{r} stride{stride} C{C}", flush=True)
    xb, gb, gl = ops.sgwls_pass_backward(direction, cuda(x), cuda(g), cuda(yb), p)
    torch.cuda.synchronize()
    rx, rg, rl = oracle.pass_backward("col" if direction == 0 else "row", x.astype(np.float64),
                                      g.astype(np.float64), yb.astype(np.float64),
                                      oracle.OracleParams(**pd))
    tag = f"dir{direction} r{r} s{stride} C{C}"
    check(f"xbar {tag}", xb.cpu().numpy(), rx, TOL_X)
    check(f"gbar {tag}", gb.cpu().numpy(), rg, TOL_G)
    check(f"lambda {tag}", gl.item(), rl, TOL_G)


@pytest.mark.parametrize("kind,prec", [("frac", "fp64_pivot"), ("exp", "fp64_pivot"),
                                       ("frac", "fp32"), ("frac", "auto"), ("exp", "auto")])
def test_pass_backward_kinds_and_precisions(ops, kind, prec):
    C, M, N = 3, 66, 140
    x, g, yb = inputs(C, M, N, 7)
    pd = pdict(lam=8.0, kind=kind)
    p = ops.Params(**pd, prec=prec)
    for direction in (0, 1):
        xb, gb, gl = ops.sgwls_pass_backward(direction, cuda(x), cuda(g), cuda(yb), p)
        torch.cuda.synchronize()
        rx, rg, rl = oracle.pass_backward("col" if direction == 0 else "row", x.astype(np.float64),
                                          g.astype(np.float64), yb.astype(np.float64),
                                          oracle.OracleParams(**pd))
        tag = f"{kind} {prec} dir{direction}"
        # frac weights in explicit float32 lose digits to cancellation (reported,
        # looser bar); the default precision takes FP64 pivots there
        tol_x = TOL_X if prec != "fp32" else 1e-3
        tol_g = TOL_G if prec != "fp32" else 1e-2
        check(f"xbar {tag}", xb.cpu().numpy(), rx, tol_x)
        check(f"gbar {tag}", gb.cpu().numpy(), rg, tol_g)
        check(f"lambda {tag}", gl.item(), rl, tol_g)


def filter_grads(ops, f, g, pd, ub, prec="auto"):
    p = ops.Params(**pd, prec=prec)
    ft, gt = cuda(f), cuda(g)
    C, M, N = f.shape
    saved = torch.empty((2 * p.iters, C, M, N), device="cuda")
    ops.sgwls_filter(ft, gt, p, saved=saved)
    gf, gg, gl = ops.sgwls_backward(gt, saved, cuda(ub), p)
    torch.cuda.synchronize()
    return gf.cpu().numpy(), gg.cpu().numpy(), gl.item()


def oracle_grads(f, g, pd, ub):
    P = oracle.OracleParams(**pd)
    _, saved = oracle.filter(f.astype(np.float64), g.astype(np.float64), P, save=True)
    return oracle.filter_backward(g.astype(np.float64), saved, ub.astype(np.float64), P)


@pytest.mark.parametrize("r,C,iters", [(1, 3, 2), (1, 1, 3), (2, 3, 1)])
def test_filter_backward_matches_oracle(ops, r, C, iters):
    M, N = 90, 130
    f, g, ub = inputs(C, M, N, 31 * r + C)
    pd = pdict(lam=8.0, r=r, iters=iters)
    gf, gg, gl = filter_grads(ops, f, g, pd, ub)
    rf, rg, rl = oracle_grads(f, g, pd, ub)
    tag = f"r{r} C{C} T{iters}"
    check(f"grad_f {tag}", gf, rf, TOL_X)
    check(f"grad_g {tag}", gg, rg, TOL_G)
    check(f"grad_lambda {tag}", gl, rl, TOL_G)


def test_filter_backward_multiwave_long_run_solver(ops):
    """700 x 300 at r = 3: the backward's long-run interface solves (six
    right-hand sides) run with four waves per strip on the column frame and
    two on the row frame."""
    M, N = 700, 300
    f, g, ub = inputs(3, M, N, 4242)
    pd = pdict(lam=8.0, r=3, iters=1)
    gf, gg, gl = filter_grads(ops, f, g, pd, ub)
    rf, rg, rl = oracle_grads(f, g, pd, ub)
    check("grad_f multi-wave long", gf, rf, TOL_X)
    check("grad_g multi-wave long", gg, rg, TOL_G)
    check("grad_lambda multi-wave long", gl, rl, TOL_G)


@pytest.mark.parametrize("r,prec", [(4, "fp32"), (3, "fp64_pivot")])
def test_filter_backward_two_wave_long_run_solver(ops, r, prec):
    """600 x 60: the column frame's ~52 strips with 299 separators each run
    the backward's long-run interface on two waves per strip (the four-wave
    exchange would pass 64 KiB of LDS at these right-hand-side counts)."""
    M, N = 600, 60
    f, g, ub = inputs(2, M, N, 4300 + r)
    pd = pdict(lam=8.0, r=r, iters=1)
    gf, gg, gl = filter_grads(ops, f, g, pd, ub, prec=prec)
    rf, rg, rl = oracle_grads(f, g, pd, ub)
    tag = f"two-wave long r{r} {prec}"
    check(f"grad_f {tag}", gf, rf, TOL_X)
    check(f"grad_g {tag}", gg, rg, TOL_G)
    if prec != "fp32":   # the float32 lambda gradient is outside the policy's bar
        check(f"grad_lambda {tag}", gl, rl, TOL_G)


@pytest.mark.parametrize("r,C", [(1, 3), (3, 1)])
def test_filter_backward_long_lines(ops, r, C):
    """Tall images (4,000 rows): more separator blocks per lane than the
    register interface solver holds, so the backward runs the scratch-backed
    solver with its doubled right-hand sides; r = 3 takes it at any length."""
    M, N = 4000, 29
    f, g, ub = inputs(C, M, N, 77 + r)
    pd = pdict(lam=8.0, r=r, iters=1)
    gf, gg, gl = filter_grads(ops, f, g, pd, ub)
    rf, rg, rl = oracle_grads(f, g, pd, ub)
    tag = f"long r{r} C{C}"
    check(f"grad_f {tag}", gf, rf, TOL_X)
    check(f"grad_g {tag}", gg, rg, TOL_G)
    check(f"grad_lambda {tag}", gl, rl, TOL_G)


@pytest.mark.parametrize("r,stride,C", [(1, 1, 3), (2, 1, 1), (1, 3, 3), (3, 1, 1)])
def test_dot_product_identity_on_gpu(ops, r, stride, C):
    """The backward is the adjoint of the forward: for the filter S (linear in
    f for a fixed guidance), <S f, v> = <f, S^T v>, both sides from the GPU
    and summed in float64."""
    M, N = 70, 95
    f, g, v = inputs(C, M, N, 500 + 10 * r + stride)
    pd = pdict(lam=5.0, r=r, iters=2, stride=stride)
    p = ops.Params(**pd)
    ft, gt = cuda(f), cuda(g)
    saved = torch.empty((2 * p.iters, C, M, N), device="cuda")
    u = ops.sgwls_filter(ft, gt, p, saved=saved)
    gf, _, _ = ops.sgwls_backward(gt, saved, cuda(v), p)
    torch.cuda.synchronize()
    lhs = float(np.sum(u.cpu().numpy().astype(np.float64) * v))
    rhs = float(np.sum(f.astype(np.float64) * gf.cpu().numpy()))
    scale = float(np.sum(np.abs(u.cpu().numpy() * v)))
    print(f"[backward] <Sf, v> {lhs:.9e} <f, S^T v> {rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_backward_of_the_differentiation_config(ops):
    """One image of the 16 x 3 x 512 x 512 differentiation workload (r=1,
    T=3, lambda=8, MSE loss to the seeded noise-free target)."""
    fs, gs, ts = synth.rgb_batch_with_target(B=1, M=512, N=512)
    f, g, tgt = fs[0], gs[0], ts[0]
    pd = pdict(lam=8.0, r=1, iters=3, sigma_r=0.1)
    P = oracle.OracleParams(**pd)
    u, saved = oracle.filter(f.astype(np.float64), g.astype(np.float64), P, save=True)
    ub = 2.0 * (u - tgt) / u.size                   # d MSE / d u
    rf, rg, rl = oracle.filter_backward(g.astype(np.float64), saved, ub, P)
    gf, gg, gl = filter_grads(ops, f, g, pd, ub.astype(np.float32))
    check("grad_f 512^2 cfg", gf, rf, TOL_X)
    check("grad_g 512^2 cfg", gg, rg, TOL_G)
    check("grad_lambda 512^2 cfg", gl, rl, TOL_G)


def test_gradients_against_finite_differences(ops):
    """GPU gradients of a 32 x 32 RGB crop against central differences of the
    FP64 oracle (h = 1e-3), for lambda, sampled guidance pixels and sampled
    input pixels; loss = sum(u * W) for a fixed random W."""
    rng = np.random.default_rng(5)
    C, M, N = 3, 32, 32
    f = rng.uniform(0, 1, (C, M, N))
    g = f.mean(axis=0) + 0.05 * rng.standard_normal((M, N))
    Wt = rng.standard_normal((C, M, N))
    pd = pdict(lam=8.0, iters=3, sigma_r=0.1)
    gf, gg, gl = filter_grads(ops, f.astype(np.float32), g.astype(np.float32), pd,
                              Wt.astype(np.float32))
    f32, g32 = f.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)

    def loss(ff, gg_, lam):
        return float((oracle.filter(ff, gg_, oracle.OracleParams(**{**pd, "lam": lam})) * Wt).sum())

    h = 1e-3
    fd_l = (loss(f32, g32, pd["lam"] + h) - loss(f32, g32, pd["lam"] - h)) / (2 * h)
    check("grad_lambda vs FD", gl, fd_l, 1e-4)
    gerr, ferr, gscale, fscale = 0.0, 0.0, np.abs(gg).max(), np.abs(gf).max()
    for (i, j) in [(0, 0), (5, 17), (16, 16), (31, 9), (20, 31), (11, 2)]:
        gp, gm = g32.copy(), g32.copy()
        gp[i, j] += h
        gm[i, j] -= h
        fd = (loss(f32, gp, pd["lam"]) - loss(f32, gm, pd["lam"])) / (2 * h)
        gerr = max(gerr, abs(gg[i, j] - fd) / gscale)
        fp, fm = f32.copy(), f32.copy()
        fp[1, i, j] += h
        fm[1, i, j] -= h
        fd = (loss(fp, g32, pd["lam"]) - loss(fm, g32, pd["lam"])) / (2 * h)
        ferr = max(ferr, abs(gf[1, i, j] - fd) / fscale)
    print(f"[backward] FD: grad_g {gerr:.3e} grad_f {ferr:.3e}", flush=True)
    assert gerr <= 1e-4 and ferr <= 1e-4


def test_backward_is_deterministic_and_accepts_aliasing(ops):
    C, M, N = 3, 80, 120
    f, g, ub = inputs(C, M, N, 77)
    pd = pdict(lam=8.0, iters=2)
    a = filter_grads(ops, f, g, pd, ub)
    b = filter_grads(ops, f, g, pd, ub)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    # grad_f may alias grad_u
    p = ops.Params(**pd)
    ft, gt = cuda(f), cuda(g)
    saved = torch.empty((2 * p.iters, C, M, N), device="cuda")
    ops.sgwls_filter(ft, gt, p, saved=saved)
    gu = cuda(ub)
    ops.sgwls_backward(gt, saved, gu, p, grad_f=gu)
    torch.cuda.synchronize()
    assert np.array_equal(gu.cpu().numpy(), a[0])


def test_autograd_function_batch(ops):
    B, C, M, N = 2, 3, 48, 64
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    g = f.mean(axis=1)
    tgt = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    pd = pdict(lam=8.0, iters=3, sigma_r=0.1)
    p = ops.Params(**pd)
    ft = cuda(f).requires_grad_(True)
    gt = cuda(g).requires_grad_(True)
    lam = torch.tensor([8.0], device="cuda", requires_grad=True)
    u = ops.sgwls(ft, gt, lam, p)
    loss = ((u - cuda(tgt)) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    gl_ref = 0.0
    for b in range(B):
        P = oracle.OracleParams(**pd)
        ub_, saved = oracle.filter(f[b].astype(np.float64), g[b].astype(np.float64), P, save=True)
        ubar = 2.0 * (ub_ - tgt[b]) / tgt.size
        rf, rg, rl = oracle.filter_backward(g[b].astype(np.float64), saved, ubar, P)
        check(f"autograd grad_f[{b}]", ft.grad[b].cpu().numpy(), rf, TOL_X)
        check(f"autograd grad_g[{b}]", gt.grad[b].cpu().numpy(), rg, TOL_G)
        gl_ref += rl
    check("autograd grad_lambda", lam.grad.item(), gl_ref, TOL_G)


def test_differentiation_workload_at_size(ops):
    """The full differentiation workload: 16 RGB 512 x 512 images, r = 1,
    T = 3, a learnable lambda = 8, loss = MSE to the seeded noise-free targets,
    forward and backward through the autograd function.  Four of the images
    are compared with the FP64 oracle's adjoint; the other twelve only enter
    the lambda gradient, whose value is checked through those four plus the
    per-image identity below."""
    B, C, M, N = 16, 3, 512, 512
    fs, gs, ts = synth.rgb_batch_with_target(B=B, M=M, N=N)
    pd = pdict(lam=8.0, r=1, iters=3, sigma_r=0.1)
    p = ops.Params(**pd)
    ft = cuda(fs).requires_grad_(True)
    gt = cuda(gs).requires_grad_(True)
    lam = torch.tensor([8.0], device="cuda", requires_grad=True)
    print("[backward] differentiation workload 16x3x512x512 through ops.sgwls", flush=True)
    u = ops.sgwls(ft, gt, lam, p)
    loss = ((u - cuda(ts)) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    P = oracle.OracleParams(**pd)
    uu = u.detach().cpu().numpy()
    total = float(ts.size)
    for b in (0, 5, 10, 15):
        ub_, saved = oracle.filter(fs[b].astype(np.float64), gs[b].astype(np.float64), P, save=True)
        check(f"cfg u[{b}]", uu[b], ub_, 1e-5)
        ubar = 2.0 * (ub_ - ts[b]) / total
        rf, rg, rl = oracle.filter_backward(gs[b].astype(np.float64), saved, ubar, P)
        check(f"cfg grad_f[{b}]", ft.grad[b].cpu().numpy(), rf, TOL_X)
        check(f"cfg grad_g[{b}]", gt.grad[b].cpu().numpy(), rg, TOL_G)
        # the batch's lambda gradient is the sum of per-image gradients: image b alone
        lb = torch.tensor([8.0], device="cuda", requires_grad=True)
        ub_gpu = ops.sgwls(cuda(fs[b]), cuda(gs[b]), lb, p)
        (((ub_gpu - cuda(ts[b])) ** 2).sum() / total).backward()
        torch.cuda.synchronize()
        check(f"cfg grad_lambda[{b}]", lb.grad.item(), rl, TOL_G)
    assert np.isfinite(lam.grad.item())


@pytest.mark.parametrize("b,i0,j0", [(0, 100, 200), (7, 300, 40), (15, 480, 480)])
def test_differentiation_crops_against_finite_differences(ops, b, i0, j0):
    """32 x 32 crops cut from images of the differentiation workload (input,
    guidance and target), run through the autograd function with MSE loss:
    the lambda gradient and sampled guidance and input gradients against
    central differences of the FP64 oracle (h = 1e-3)."""
    fs, gs, ts = synth.rgb_batch_with_target(B=b + 1, M=512, N=512)
    f = fs[b][:, i0:i0 + 32, j0:j0 + 32].astype(np.float64)
    g = gs[b][i0:i0 + 32, j0:j0 + 32].astype(np.float64)
    t = ts[b][:, i0:i0 + 32, j0:j0 + 32].astype(np.float64)
    pd = pdict(lam=8.0, r=1, iters=3, sigma_r=0.1)
    p = ops.Params(**pd)
    ft = cuda(f).requires_grad_(True)
    gt = cuda(g).requires_grad_(True)
    lam = torch.tensor([8.0], device="cuda", requires_grad=True)
    u = ops.sgwls(ft, gt, lam, p)
    ((u - cuda(t)) ** 2).mean().backward()
    torch.cuda.synchronize()
    gf, gg, gl = ft.grad.cpu().numpy(), gt.grad.cpu().numpy(), lam.grad.item()
    f32, g32 = f.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)

    def loss(ff, gg_, lm):
        return float(((oracle.filter(ff, gg_, oracle.OracleParams(**{**pd, "lam": lm})) - t) ** 2).mean())

    h = 1e-3
    fd_l = (loss(f32, g32, 8.0 + h) - loss(f32, g32, 8.0 - h)) / (2 * h)
    check(f"crop{b} grad_lambda vs FD", gl, fd_l, 1e-4)
    gerr, ferr, gscale, fscale = 0.0, 0.0, np.abs(gg).max(), np.abs(gf).max()
    for (i, j) in [(0, 0), (7, 21), (16, 16), (31, 3), (24, 31)]:
        gp, gm = g32.copy(), g32.copy()
        gp[i, j] += h
        gm[i, j] -= h
        gerr = max(gerr, abs(gg[i, j] - (loss(f32, gp, 8.0) - loss(f32, gm, 8.0)) / (2 * h)) / gscale)
        fp, fm = f32.copy(), f32.copy()
        fp[2, i, j] += h
        fm[2, i, j] -= h
        ferr = max(ferr, abs(gf[2, i, j] - (loss(fp, g32, 8.0) - loss(fm, g32, 8.0)) / (2 * h)) / fscale)
    print(f"[backward] crop{b} FD: grad_g {gerr:.3e} grad_f {ferr:.3e}", flush=True)
    assert gerr <= 1e-4 and ferr <= 1e-4
