"""Backward with saved separators (sgwls_filter_nchw_seps, then
sgwls_backward_nchw_seps) against the FP64 CPU oracle's adjoint, and against
the plain forward/backward pair at the full differentiation workload.

The forward keeps every pass's solution at the separators of the backward's
chunks (stored by its re-solve, whatever its own chunks); each backward pass
then eliminates only the adjoint's right-hand sides and re-solves both with
the forward's separators.
Same tolerances as the plain backward: the arithmetic per chunk is the same,
in the same precision.  Error measure: normwise relative, max|gpu - ref| /
max|ref|.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle

pytestmark = pytest.mark.gpu

TOL_X = 1e-5
TOL_G = 1e-4


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def check(name, gpu, ref, tol):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mx = np.abs(gpu - ref).max() / max(np.abs(ref).max(), 1e-300)
    print(f"[seps] {name}: max {mx:.3e}", flush=True)
    assert mx <= tol, f"{name}: {mx:.3e} > {tol:.1e}"


def pdict(lam, r, iters, sigma_r=0.2):
    return dict(lam=lam, r=r, iters=iters, stride=1, kind="exp", sigma_s=float(r),
                sigma_r=sigma_r, alpha_s=1.2, alpha_r=1.2, eps=1e-4)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run_seps(ops, f, g, ub, p):
    B, C, M, N = f.shape
    nsep = ops.separator_bytes_nchw(B, C, M, N, p)
    assert nsep > 0
    seps = torch.empty(nsep, dtype=torch.uint8, device="cuda")
    saved = torch.empty((B, 2 * p.iters, C, M, N), device="cuda")
    lam = torch.tensor([p.lam], device="cuda")
    ft = cuda(f)
    u = ops.sgwls_filter_nchw(ft, cuda(g), p, lambda_dev=lam, saved=saved, seps=seps)
    gf, gg, gl = ops.sgwls_backward_nchw(cuda(g), saved, cuda(ub), p, lambda_dev=lam, seps=seps,
                                         f=ft)
    torch.cuda.synchronize()
    return u.cpu().numpy(), gf.cpu().numpy(), gg.cpu().numpy(), gl.item()


# Cases: both precisions, r = 1..4, one and three channels, four channels
# (a three-channel block and a single channel), batches, several chunks and
# ragged edges in both frames.
CASES = [
    (1, 3, 70, 150, 1, "fp32", 1),
    (2, 3, 70, 150, 1, "fp64_pivot", 2),
    (1, 1, 90, 130, 1, "fp32", 2),
    (1, 1, 90, 130, 1, "fp64_pivot", 1),
    (1, 1, 90, 130, 2, "fp32", 1),
    (2, 3, 66, 98, 2, "fp32", 1),
    (1, 3, 66, 98, 2, "fp64_pivot", 1),
    (1, 4, 60, 140, 1, "fp32", 2),
    (1, 3, 50, 90, 3, "fp32", 1),
    (1, 1, 60, 80, 4, "fp64_pivot", 1),
    (1, 3, 44, 70, 4, "fp32", 1),
    # edges: one chunk per column (no separators in that frame), the
    # minimum height 2r+1 (one strip in the row frame), five channels (blocks
    # 3, 1, 1), and lines long enough for the scratch-backed long-run
    # interface (more than 512 separators) in the forward and the adjoint
    (1, 2, 5, 200, 1, "fp32", 1),
    (1, 3, 3, 64, 1, "fp64_pivot", 1),
    (1, 5, 40, 90, 1, "fp64_pivot", 1),
    (1, 3, 3300, 40, 1, "fp32", 1),
    (1, 1, 40, 2100, 2, "fp32", 1),
    # forward chunks taller than the backward's (separators stored from
    # inside the forward's chunks): r = 3 grey in float32, r = 2 grey with
    # FP64 pivots
    (1, 1, 70, 110, 3, "fp32", 1),
    (1, 1, 66, 98, 2, "fp64_pivot", 2),
    # the same stores in a batch (per-image offsets), and four channels at
    # r = 3 (the three-channel block through the interface, the single
    # channel through the re-solve, in one call)
    (2, 1, 58, 84, 3, "fp32", 1),
    (1, 4, 50, 90, 3, "fp32", 1),
]


@pytest.mark.parametrize("B,C,M,N,r,prec,iters", CASES)
def test_seps_backward_matches_oracle(ops, B, C, M, N, r, prec, iters):
    print(f"[seps] B{B} C{C} {M}x{N} r{r} {prec} T{iters}", flush=True)
    rng = np.random.default_rng(1000 * r + 10 * C + M + iters)
    f = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    g = rng.uniform(0, 1, (B, M, N)).astype(np.float32)
    ub = rng.standard_normal((B, C, M, N)).astype(np.float32)
    pd = pdict(lam=6.0, r=r, iters=iters)
    p = ops.Params(**pd, prec=prec)
    u, gf, gg, gl = run_seps(ops, f, g, ub, p)
    P = oracle.OracleParams(**pd)
    gl_ref = 0.0
    for b in range(B):
        ru, saved = oracle.filter(f[b].astype(np.float64), g[b].astype(np.float64), P, save=True)
        rf, rg, rl = oracle.filter_backward(g[b].astype(np.float64), saved,
                                            ub[b].astype(np.float64), P)
        check(f"u[{b}]", u[b], ru, TOL_X)
        check(f"grad_f[{b}]", gf[b], rf, TOL_X)
        check(f"grad_g[{b}]", gg[b], rg, TOL_G)
        gl_ref += rl
    check("grad_lambda", gl, gl_ref, TOL_G)


@pytest.mark.parametrize("prec", ["fp64_pivot", "fp32"])
def test_seps_pair_matches_plain_pair_at_1080p(ops, prec):
    # The differentiation workload: 1080 x 1920 RGB, r = 1, T = 3.
    B, C, M, N = 1, 3, 1080, 1920
    print(f"[seps] 1080p RGB r1 T3 {prec}", flush=True)
    rng = np.random.default_rng(77)
    f = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    g = f.mean(axis=1)
    ub = rng.standard_normal((B, C, M, N)).astype(np.float32)
    p = ops.Params(**pdict(lam=4.0, r=1, iters=3, sigma_r=0.1), prec=prec)
    u, gf, gg, gl = run_seps(ops, f, g, ub, p)
    saved = torch.empty((B, 6, C, M, N), device="cuda")
    lam = torch.tensor([p.lam], device="cuda")
    u0 = ops.sgwls_filter_nchw(cuda(f), cuda(g), p, lambda_dev=lam, saved=saved)
    gf0, gg0, gl0 = ops.sgwls_backward_nchw(cuda(g), saved, cuda(ub), p, lambda_dev=lam)
    torch.cuda.synchronize()
    # both pairs round differently from the exact result; against each other
    # they agree to twice the oracle tolerances
    check("u 1080p", u, u0.cpu().numpy(), 2 * TOL_X)
    check("grad_f 1080p", gf, gf0.cpu().numpy(), 2 * TOL_X)
    check("grad_g 1080p", gg, gg0.cpu().numpy(), 2 * TOL_G)
    check("grad_lambda 1080p", gl, gl0.item(), 2 * TOL_G)


def test_autograd_with_and_without_seps(ops, monkeypatch):
    B, C, M, N = 2, 3, 48, 64
    rng = np.random.default_rng(8)
    f = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    g = f.mean(axis=1)
    tgt = rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)
    p = ops.Params(**pdict(lam=8.0, r=1, iters=2, sigma_r=0.1))
    grads = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SGWLS_SAVE_SEPARATORS", flag)
        ft = cuda(f).requires_grad_(True)
        gt = cuda(g).requires_grad_(True)
        lam = torch.tensor([8.0], device="cuda", requires_grad=True)
        loss = ((ops.sgwls(ft, gt, lam, p) - cuda(tgt)) ** 2).mean()
        loss.backward()
        torch.cuda.synchronize()
        grads.append((ft.grad.cpu().numpy(), gt.grad.cpu().numpy(), lam.grad.item()))
    check("autograd grad_f", grads[0][0], grads[1][0], 2 * TOL_X)
    check("autograd grad_g", grads[0][1], grads[1][1], 2 * TOL_G)
    check("autograd grad_lambda", grads[0][2], grads[1][2], 2 * TOL_G)
