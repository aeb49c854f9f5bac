"""Right-preconditioned GMRES (oracle), Sec. 2.3: solve (A P) y = b, u = P y.

Textbook Arnoldi with modified Gram-Schmidt; after every step the small least-squares
problem min || beta e_1 - H_k z || is solved directly with numpy.linalg.lstsq, and its
residual norm is the GMRES residual.  Starting guess zero, no restart.  Stops when the
residual is reduced by the factor `tol` (the paper's criterion, Sec. 3: reduction of
the residual by 1e-6).  The iteration count is the number of operator applications.
"""
from __future__ import annotations

import numpy as np


def gmres_right(apply_op, b: np.ndarray, tol: float = 1e-6, maxit: int = 200):
    """Returns (y, iters, history) with history[k] = ||b - Op y_k|| / ||b||."""
    shape = b.shape
    bvec = b.ravel().astype(np.complex128)
    beta = np.linalg.norm(bvec)
    hist = [1.0]
    if beta == 0.0:
        return np.zeros(shape, dtype=np.complex128), 0, hist
    V = [bvec / beta]
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    z = np.zeros(0, dtype=np.complex128)
    k = 0
    for k in range(1, maxit + 1):
        w = apply_op(V[k - 1].reshape(shape)).ravel().astype(np.complex128)
        for i in range(k):                       # modified Gram-Schmidt
            H[i, k - 1] = np.vdot(V[i], w)
            w = w - H[i, k - 1] * V[i]
        H[k, k - 1] = np.linalg.norm(w)
        rhs = np.zeros(k + 1, dtype=np.complex128)
        rhs[0] = beta
        Hk = H[:k + 1, :k]
        z = np.linalg.lstsq(Hk, rhs, rcond=None)[0]
        res = np.linalg.norm(rhs - Hk @ z) / beta
        hist.append(float(res))
        if res <= tol or H[k, k - 1] == 0.0:
            break
        V.append(w / H[k, k - 1])
    y = sum(z[i] * V[i] for i in range(len(z)))
    return y.reshape(shape), k, hist
