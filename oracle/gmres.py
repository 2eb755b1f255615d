"""Right-preconditioned flexible GMRES (oracle side; test infrastructure).

Paper Sec. 5 preconditions GMRES with the HBS inverse M of the 4th-order
operator and iterates on the high-order operator applied by FFT.  Reading
used here: right preconditioning with the flexible variant (z_j = M v_j is
stored), x0 = 0, no restart, classical Gram-Schmidt applied twice, Givens
rotations on the Hessenberg matrix; the monitored quantity is the relative
residual ||f - A x_j|| / ||f||, which for right preconditioning equals the
least-squares residual |g_{j+1}| / ||f|| in exact arithmetic.
"""
from __future__ import annotations

import numpy as np


def fgmres(matvec, precond, f, tol=1e-10, maxit=100):
    f = np.asarray(f, dtype=complex).reshape(-1)
    beta = np.linalg.norm(f)
    if beta == 0:
        return np.zeros_like(f), 0, [0.0]
    V = [f / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit), dtype=complex)
    cs = np.zeros(maxit, dtype=complex)
    sn = np.zeros(maxit, dtype=complex)
    g = np.zeros(maxit + 1, dtype=complex)
    g[0] = beta
    hist = [1.0]
    j = 0
    for j in range(maxit):
        z = precond(V[j])
        Z.append(z)
        w = matvec(z)
        Vm = np.array(V)
        h = Vm.conj() @ w
        w = w - Vm.T @ h
        h2 = Vm.conj() @ w
        w = w - Vm.T @ h2
        h = h + h2
        hn = np.linalg.norm(w)
        H[: j + 1, j] = h
        H[j + 1, j] = hn
        V.append(w / hn if hn > 0 else w)
        for i in range(j):
            a, c = H[i, j], H[i + 1, j]
            H[i, j] = np.conj(cs[i]) * a + np.conj(sn[i]) * c
            H[i + 1, j] = -sn[i] * a + cs[i] * c
        a, c = H[j, j], H[j + 1, j]
        rho = np.hypot(abs(a), abs(c))
        cs[j] = a / rho if rho else 1.0
        sn[j] = c / rho if rho else 0.0
        H[j, j] = rho
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = np.conj(cs[j]) * g[j]
        hist.append(abs(g[j + 1]) / beta)
        if hist[-1] < tol or hn == 0:
            break
    k = j + 1
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = np.array(Z).T @ y
    return x, k, hist
