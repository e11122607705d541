"""Outer iterations around the V-cycle, FP64 (oracle side).

The paper uses the V-cycle as a stationary solver and as a preconditioner for
CG (symmetric problems) and GMRES (Section 5), stopping when
||f - A u|| / ||f|| < tol from u = 0.  Readings: the preconditioner is applied
on the right for GMRES so that the stopping test is on the true residual; the
Arnoldi basis is orthogonalised by classical Gram-Schmidt applied twice (CGS2);
the relative residual is always the true one, recomputed in FP64 whenever the
recurrence says the tolerance is met.
"""
import numpy as np
import scipy.linalg as sla


def stationary(A, b, M, tol, maxit, x0=None):
    """x <- x + M(b - A x) (Algorithm 2's outer loop, correction form)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    hist = []
    for it in range(1, maxit + 1):
        x = x + M(b - A @ x)
        rel = np.linalg.norm(b - A @ x) / nb
        hist.append(rel)
        if rel <= tol:
            return x, it, hist
    return x, maxit, hist


def pcg(A, b, M, tol, maxit, x0=None):
    """Preconditioned conjugate gradients (Hestenes-Stiefel) with M ~ A^{-1}.

    The recursive residual decides when to look; the true residual decides when
    to stop.  Returns (x, iterations, history of recursive relative residuals)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    if np.linalg.norm(r) <= tol * nb:
        return x, 0, []
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = []
    for it in range(1, maxit + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0:
            raise FloatingPointError("pCG breakdown: p^T A p <= 0")
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol and np.linalg.norm(b - A @ x) / nb <= tol:
            return x, it, hist
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def fgmres(A, b, M, tol, restart, maxit, x0=None):
    """Restarted flexible GMRES with right preconditioning (z_j = M(v_j) stored),
    CGS2 Arnoldi and Givens rotations.  Every restart starts from the true FP64
    residual, so with an inexact (e.g. lower-precision) M this is iterative
    refinement with an FGMRES inner solver.  Returns (x, iterations, history)."""
    n = len(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    total = 0
    hist = []
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * nb or total >= maxit:
            return x, total, hist
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = A @ Z[j]
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or total >= maxit:
                break
        y = sla.solve_triangular(H[:j_end, :j_end], g[:j_end])
        x = x + Z[:j_end].T @ y


def fcg(A, b, M, tol, maxit, x0=None, replace_drop=1e-6):
    """Flexible preconditioned CG (Polak-Ribiere form of beta,
    beta = z_new^T (r_new - r_old) / (z_old^T r_old)), for a preconditioner M that
    is only approximately symmetric (e.g. a V-cycle evaluated in lower precision).

    Residual replacement: whenever the recursive residual claims convergence, or
    has dropped by ``replace_drop`` since the last replacement, the true FP64
    residual b - A x is computed; if it does not meet the tolerance it replaces
    the recursive one (the search direction is kept).  With a low-precision M
    this keeps the recursive residual from drifting away from the true one, so
    the tolerance stays attainable.  Returns (x, iterations, history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    anchor = np.linalg.norm(r) / nb
    if anchor <= tol:
        return x, 0, []
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = []
    for it in range(1, maxit + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0:
            raise FloatingPointError("fCG breakdown: p^T A p <= 0")
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol or rel <= anchor * replace_drop:
            rt = b - A @ x
            true_rel = np.linalg.norm(rt) / nb
            if true_rel <= tol:
                return x, it, hist
            r, anchor = rt, true_rel
        z = M(r)
        beta = (z @ (r - r_old)) / rz
        rz = r @ z
        p = z + beta * p
    return x, maxit, hist
