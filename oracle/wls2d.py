"""The 2D WLS model the paper approximates (Eqs. 1-4), solved exactly in
FP64 on the CPU.

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU conjugate-
gradient solver of the same model; only ``tests/`` imports it.  It shares no
code with the GPU library.

Model: U minimises sum_i (u_i - f_i)^2 + lambda * sum over unordered pixel
pairs {i, j} with j in the (2r+1) x (2r+1) patch around i of
omega_ij (u_i - u_j)^2, i.e. (I + lambda L) U = F (Eq. 4 with the pairs of
the square patch, Eq. 1), per channel.  omega_ij is Eq. 2 with |i - j| the
Euclidean distance between the two pixel positions.  The matrix is assembled
term by term and handed to a sparse direct solver (scipy's spsolve).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def weight(params, dist: float, gi: np.ndarray, gj: np.ndarray) -> np.ndarray:
    """omega of Eq. 2 for pixel pairs at Euclidean distance dist."""
    d = gi - gj
    if params.kind == "exp":
        return math.exp(-dist * dist / (2.0 * params.sigma_s ** 2)) * np.exp(
            -d * d / (2.0 * params.sigma_r ** 2))
    return (1.0 / (dist ** params.alpha_s + params.eps)) / (np.abs(d) ** params.alpha_r + params.eps)


def matrix(g: np.ndarray, params) -> sp.csr_matrix:
    """A = I + lambda L over the (2r+1)^2 patch pairs (Eq. 4)."""
    g = np.asarray(g, dtype=np.float64)
    M, N = g.shape
    r = params.r
    idx = np.arange(M * N).reshape(M, N)
    rows, cols, vals = [], [], []
    diag = np.ones(M * N)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy == 0 and dx == 0:
                continue
            # pixels i = (y, x) whose neighbour j = (y + dy, x + dx) is inside
            yi = slice(max(0, -dy), M - max(0, dy))
            xi = slice(max(0, -dx), N - max(0, dx))
            yj = slice(max(0, dy), M - max(0, -dy))
            xj = slice(max(0, dx), N - max(0, -dx))
            w = params.lam * weight(params, math.hypot(dy, dx), g[yi, xi], g[yj, xj])
            i, j = idx[yi, xi].ravel(), idx[yj, xj].ravel()
            rows.append(i)
            cols.append(j)
            vals.append(-w.ravel())
            np.add.at(diag, i, w.ravel())
    rows.append(np.arange(M * N))
    cols.append(np.arange(M * N))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(M * N, M * N))


def wls2d(F: np.ndarray, g: np.ndarray, params) -> np.ndarray:
    """Exact 2D WLS output of F ((C, M, N) or (M, N)) with guidance g."""
    F = np.asarray(F, dtype=np.float64)
    sq = F.ndim == 2
    F3 = F[None] if sq else F
    C, M, N = F3.shape
    A = matrix(g, params).tocsc()
    lu = spla.splu(A)
    U = np.stack([lu.solve(F3[c].ravel()).reshape(M, N) for c in range(C)])
    return U[0] if sq else U


def energy(U: np.ndarray, F: np.ndarray, g: np.ndarray, params) -> float:
    """The objective of Eq. 1 as a plain sum over pixels and over unordered
    neighbour pairs (each pair once), for pinning the assembly."""
    U = np.asarray(U, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    M, N = g.shape
    r = params.r
    e = float(((U - F) ** 2).sum())
    for y in range(M):
        for x in range(N):
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    yy, xx = y + dy, x + dx
                    if (dy, dx) <= (0, 0) or not (0 <= yy < M and 0 <= xx < N):
                        continue   # each unordered pair once: the later pixel
                    w = float(weight(params, math.hypot(dy, dx), np.array(g[y, x]),
                                     np.array(g[yy, xx])))
                    e += params.lam * w * (U[y, x] - U[yy, xx]) ** 2
    return e
