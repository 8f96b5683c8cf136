"""Pins of the 2D WLS oracle (Eqs. 1-4) against what the model fixes
independently of the assembled matrix: the minimiser of the objective
(written as a plain sum over unordered pairs) has zero gradient, the
gradient of that objective is 2((I + lambda L) U - F), constants pass
through, lambda = 0 is the identity, the matrix is a symmetric M-matrix with
unit row sums, and the output obeys the maximum principle."""
import numpy as np
import pytest

import oracle
from oracle import wls2d as W


def params(kind="exp", r=1, lam=3.0):
    return oracle.OracleParams(lam=lam, r=r, iters=1, stride=1, kind=kind, sigma_s=float(r),
                               sigma_r=0.3, alpha_s=1.2, alpha_r=1.2, eps=1e-2)


def fd_grad(U, F, g, P, h=1e-6):
    G = np.zeros_like(U)
    for i in range(U.shape[0]):
        for j in range(U.shape[1]):
            Up, Um = U.copy(), U.copy()
            Up[i, j] += h
            Um[i, j] -= h
            G[i, j] = (W.energy(Up, F, g, P) - W.energy(Um, F, g, P)) / (2 * h)
    return G


@pytest.mark.parametrize("kind", ["exp", "frac"])
@pytest.mark.parametrize("r", [1, 2])
def test_solution_minimises_the_objective(kind, r):
    rng = np.random.default_rng(10 * r + (kind == "frac"))
    g = rng.uniform(0, 1, (5, 6))
    F = rng.normal(size=(5, 6))
    P = params(kind, r)
    U = W.wls2d(F, g, P)
    assert np.abs(fd_grad(U, F, g, P)).max() <= 1e-5 * max(1.0, np.abs(F).max())
    # at an arbitrary point the objective's gradient is 2 (A V - F)
    V = rng.normal(size=(5, 6))
    A = W.matrix(g, P)
    want = 2.0 * (A @ V.ravel() - F.ravel()).reshape(5, 6)
    assert np.abs(fd_grad(V, F, g, P) - want).max() <= 1e-5 * np.abs(want).max()


@pytest.mark.parametrize("kind", ["exp", "frac"])
def test_matrix_structure_and_invariants(kind):
    rng = np.random.default_rng(3)
    g = rng.uniform(0, 1, (9, 7))
    P = params(kind, 2, lam=5.0)
    A = W.matrix(g, P).toarray()
    assert np.abs(A - A.T).max() <= 1e-12
    assert np.abs(A.sum(axis=1) - 1.0).max() <= 1e-9
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0.0
    assert (off < 0).sum(axis=1).max() == 24        # the full 5 x 5 patch inside
    F = rng.uniform(-1, 2, (2, 9, 7))
    U = W.wls2d(F, g, P)
    assert U.min() >= F.min() - 1e-12 and U.max() <= F.max() + 1e-12
    assert np.abs(W.wls2d(np.full((9, 7), 0.7), g, P) - 0.7).max() <= 1e-12
    assert np.abs(W.wls2d(F, g, params(kind, 2, lam=0.0)) - F).max() <= 1e-14
