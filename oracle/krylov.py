"""Flexible GMRES (oracle; test infrastructure only).

Section 3.3 uses GMRES as the outer solver with the multigrid
preconditioner.  Reading: right-preconditioned flexible GMRES(m)
(Saad, Iterative Methods, Alg. 9.6) with classical Gram-Schmidt applied
twice, Givens rotations, x0 = 0.  A cycle ends when the Givens estimate
of the residual drops to rtol * ||b||; the solve ends when the explicit
residual ||b - A x|| confirms it, otherwise it restarts from x.
"""
import numpy as np


def givens(a, b):
    """(c, s) with [c s; -s c] [a; b] = [r; 0]."""
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(A, M, b, m=30, rtol=1e-8, max_iter=300):
    """Returns (x, info) with info = dict(iterations, converged, rel_residual)."""
    n = b.size
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, dict(iterations=0, converged=True, rel_residual=0.0)
    it = 0
    while True:
        r = b - A(x)
        beta = float(np.linalg.norm(r))
        if beta <= rtol * bnorm:
            return x, dict(iterations=it, converged=True, rel_residual=beta / bnorm)
        if it >= max_iter:
            return x, dict(iterations=it, converged=False, rel_residual=beta / bnorm)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        jend = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            h1 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h1
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            H[: j + 1, j] = h1 + h2
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            jend = j + 1
            if abs(g[j + 1]) <= rtol * bnorm or it >= max_iter or hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: jend] @ y[i + 1:]) / H[i, i]
        x = x + Z[:jend].T @ y
