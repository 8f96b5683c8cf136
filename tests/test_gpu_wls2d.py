"""The GPU conjugate-gradient solver of the 2D WLS model (Eqs. 1-4) against
the exact FP64 solve of the oracle, and the SG-WLS approximation gap it
measures.

Error measure: normwise relative, max|gpu - oracle| / max|oracle|.  Bar:
1e-5 with the solver run to a relative residual of 1e-7 (the error is at
most the condition number times the residual; float32 vectors)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import wls2d as W
from paper_1705_01674_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01674_amd import ops as _ops
    return _ops


def pd(kind="exp", r=1, lam=4.0, sigma_r=0.1):
    return dict(lam=lam, r=r, iters=1, stride=1, kind=kind, sigma_s=float(r), sigma_r=sigma_r,
                alpha_s=1.2, alpha_r=1.2, eps=1e-2)


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / np.abs(b).max())


@pytest.mark.parametrize("kind,r,lam", [("exp", 1, 4.0), ("exp", 2, 10.0), ("exp", 4, 2.0),
                                        ("frac", 1, 0.5), ("frac", 3, 0.2)])
@pytest.mark.parametrize("C", [1, 3])
def test_cg_matches_exact_solve(ops, kind, r, lam, C):
    img = synth.image(70, 83, 3, 20, 0.03, seed=3000 + r)
    f = np.ascontiguousarray(img[:C])
    g = synth.luma(img)
    d = pd(kind, r, lam)
    u, its, res = ops.wls2d(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(),
                            ops.Params(**d), max_iters=4000, tol=1e-7)
    torch.cuda.synchronize()
    ref = W.wls2d(f.astype(np.float64), g.astype(np.float64), oracle.OracleParams(**d))
    e = rel(u.cpu().numpy(), ref)
    print(f"[wls2d] {kind} r{r} lam{lam} C{C}: {its} iterations, residual {res:.2e}, "
          f"error {e:.3e}", flush=True)
    assert res <= 1e-7 and e <= TOL


def test_cg_invariants(ops):
    img = synth.image(40, 50, 1, 10, 0.03, seed=3100)
    g = torch.from_numpy(synth.luma(img)).cuda()
    const = torch.full((1, 40, 50), 0.7, device="cuda")
    u, _, _ = ops.wls2d(const, g, ops.Params(**pd()), tol=1e-7)
    assert float((u - 0.7).abs().max()) <= 1e-6
    f = torch.from_numpy(img).cuda()
    u, its, _ = ops.wls2d(f, g, ops.Params(**pd(lam=0.0)), tol=1e-7)
    assert its <= 8 and float((u - f).abs().max()) <= 1e-6


def test_sgwls_approximation_gap(ops):
    """SG-WLS against the 2D WLS it approximates, both on the GPU, r = 1 and
    2, T = 3: the relative gap is reported (quality context, not parity)."""
    w = synth.rgb768x1024()
    f = torch.from_numpy(w.f).cuda()
    g = torch.from_numpy(w.g).cuda()
    for r in (1, 2):
        d = dict(w.params, r=r, sigma_s=float(r))
        sg = ops.sgwls_filter(f, g, ops.Params(**d))
        ref, its, res = ops.wls2d(f, g, ops.Params(**d), max_iters=3000, tol=1e-6)
        torch.cuda.synchronize()
        gap = float((sg - ref).abs().max() / ref.abs().max())
        mean = float((sg - ref).abs().mean() / ref.abs().max())
        print(f"[wls2d] gap r{r}: max {gap:.3e} mean {mean:.3e} ({its} CG iterations)",
              flush=True)
        assert res <= 1e-6 and gap < 0.5
