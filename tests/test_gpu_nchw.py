"""NCHW batches (every launch covers B equal-shape images, blockIdx.z =
image) against one call per image: the outputs, the saved pass inputs and
the input and guidance gradients are bitwise equal (the same kernels on the
same data), and the batch's lambda gradient is the sum of the per-image
ones (summed in another order: float64 rounding only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


@pytest.mark.parametrize("B,C,M,N,r,stride,prec", [
    (3, 3, 70, 90, 1, 1, "fp32"), (2, 1, 64, 80, 2, 3, "fp32"), (2, 4, 50, 61, 1, 1, "fp32"),
    (3, 3, 40, 52, 1, 2, "fp64_pivot"), (2, 3, 33, 47, 3, 1, "fp32"),
])
def test_nchw_equals_per_image_calls(ops, B, C, M, N, r, stride, prec):
    rng = np.random.default_rng(B * 100 + C * 10 + r + stride)
    f = torch.from_numpy(rng.uniform(0, 1, (B, C, M, N)).astype(np.float32)).cuda()
    g = torch.from_numpy(rng.uniform(0, 1, (B, M, N)).astype(np.float32)).cuda()
    yb = torch.from_numpy(rng.standard_normal((B, C, M, N)).astype(np.float32)).cuda()
    p = ops.Params(lam=5.0, r=r, iters=2, stride=stride, sigma_r=0.2, prec=prec)
    T2 = 2 * p.iters
    print(f"[nchw] B{B} C{C} {M}x{N} r{r} s{stride} {prec}", flush=True)
    saved = torch.empty((B, T2, C, M, N), device="cuda")
    u = ops.sgwls_filter_nchw(f, g, p, saved=saved)
    gf, gg, gl = ops.sgwls_backward_nchw(g, saved, yb, p)
    u_nosave = ops.sgwls_filter_nchw(f, g, p)
    torch.cuda.synchronize()
    lam_sum = 0.0
    for b in range(B):
        sb = torch.empty((T2, C, M, N), device="cuda")
        ub = ops.sgwls_filter(f[b], g[b], p, saved=sb)
        ub_nosave = ops.sgwls_filter(f[b], g[b], p)
        gfb, ggb, glb = ops.sgwls_backward(g[b], sb, yb[b].contiguous(), p)
        torch.cuda.synchronize()
        assert torch.equal(u[b], ub)
        assert torch.equal(u_nosave[b], ub_nosave)
        assert torch.equal(saved[b], sb)
        assert torch.equal(gf[b], gfb)
        assert torch.equal(gg[b], ggb)
        lam_sum += glb.item()
    assert abs(gl.item() - lam_sum) <= 1e-12 * max(abs(lam_sum), 1e-300) + 1e-15
