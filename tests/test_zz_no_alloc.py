"""sgwls_filter_noalloc (the filter with its workspace in the library's static
device array) against sgwls_filter with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller image, each bitwise equal to
the workspace call (the same kernels in the same order), plus the size limit
(refused before anything is enqueued)."""
import ctypes

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


def noalloc(ops, f, g, p, saved=None):
    nat = ops.nat
    C, M, N = f.shape
    u = torch.empty_like(f)
    st = nat.lib.sgwls_filter_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr()), C, M, N, ctypes.byref(p.c()),
                                      None, None if saved is None else ctypes.c_void_p(saved.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, u


def test_noalloc_matches_the_workspace_entry_point_twice(ops):
    rng = np.random.default_rng(17)
    for (C, M, N, r) in ((3, 1080, 1920, 1), (3, 301, 517, 2)):     # the second call is smaller
        f = torch.from_numpy(rng.uniform(0, 1, (C, M, N)).astype(np.float32)).cuda()
        g = torch.from_numpy(rng.uniform(0, 1, (M, N)).astype(np.float32)).cuda()
        p = ops.Params(lam=4.0, r=r, iters=3, sigma_r=0.1)
        print(f"[noalloc] C{C} {M}x{N} r{r}", flush=True)
        st, u = noalloc(ops, f, g, p)
        ref = ops.sgwls_filter(f, g, p)
        torch.cuda.synchronize()
        assert st == 0
        assert torch.equal(u, ref)


def test_noalloc_refuses_images_beyond_its_array(ops):
    f = torch.zeros((3, 2160, 3840), device="cuda")
    g = torch.zeros((2160, 3840), device="cuda")
    p = ops.Params(lam=4.0, r=1, iters=1)
    st, _ = noalloc(ops, f, g, p)
    assert st == 3        # SGWLS_E_WORKSPACE, nothing enqueued
