"""Textbook Krylov solvers in FP64 and the condition-number estimate.

The paper solves with "iterative solvers" and an inner conjugate gradient
(Sec. I, Sec. III code description), and measures condition numbers of the
"square operators" Mt^dagger Mt with a Ritz technique (Sec. III).  Here:

* cgnr     - Hestenes-Stiefel CG on the normal equations A^dagger A x = A^dagger b;
* bicgstab - van der Vorst's BiCGStab (1992);
* lanczos_kappa - extreme eigenvalues of the Lanczos tridiagonal matrix that CG
  builds implicitly: diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal
  sqrt(beta_k)/alpha_k.  Its ratio estimates kappa(A^dagger A).

Inner products are plain np.vdot over all components (global l2 norm).
"""
import numpy as np


def _dot(a, b):
    return np.vdot(a, b)


def _nrm2(a):
    return float(np.vdot(a, a).real)


def cgnr(A, Adag, b, tol=1e-10, maxiter=100000, x0=None):
    """Solve A x = b via CG on A^dagger A; stop on ||b - A x|| <= tol ||b||.

    Returns x, info with the residual history and the CG coefficients."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    z = Adag(r)
    p = z.copy()
    zz = _nrm2(z)
    bn = np.sqrt(_nrm2(b))
    alphas, betas = [], []
    k = 0
    res = np.sqrt(_nrm2(r)) / bn
    while res > tol and k < maxiter:
        w = A(p)
        alpha = zz / _nrm2(w)
        x = x + alpha * p
        r = r - alpha * w
        z = Adag(r)
        zz_new = _nrm2(z)
        beta = zz_new / zz
        p = z + beta * p
        zz = zz_new
        alphas.append(alpha)
        betas.append(beta)
        k += 1
        res = np.sqrt(_nrm2(r)) / bn
    return x, dict(iters=k, rel_resid=res, alphas=alphas, betas=betas)


def lanczos_kappa(alphas, betas):
    """(lambda_min, lambda_max, kappa) of A^dagger A from CG's alpha, beta."""
    n = len(alphas)
    if n == 0:
        return np.nan, np.nan, np.nan
    d = np.empty(n)
    off = np.empty(max(n - 1, 0))
    for k in range(n):
        d[k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k < n - 1:
            off[k] = np.sqrt(betas[k]) / alphas[k]
    t = np.diag(d) + np.diag(off, 1) + np.diag(off, -1)
    ev = np.linalg.eigvalsh(t)
    return ev[0], ev[-1], ev[-1] / ev[0]


def bicgstab(A, b, tol=1e-10, maxiter=100000, x0=None):
    """van der Vorst's BiCGStab; stop on ||b - A x|| <= tol ||b|| (recursive residual)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    bn = np.sqrt(_nrm2(b))
    res = np.sqrt(_nrm2(r)) / bn
    k = 0
    while res > tol and k < maxiter:
        rho_new = _dot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho_new / _dot(rhat, v)
        s = r - alpha * v
        t = A(s)
        omega = _dot(t, s) / _dot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        k += 1
        res = np.sqrt(_nrm2(r)) / bn
    return x, dict(iters=k, rel_resid=res)


def solve(op, scheme, eta, solver="bicgstab", tol=1e-10, maxiter=100000):
    """x with ||eta - M x|| / ||eta|| <= tol via eta~ = S_L eta, Mt y = eta~, x = S_R y.

    The preconditioned system is solved to a tolerance scaled by ||eta||/||eta~||
    and re-solved (restarted from the current y) until the true residual of the
    original system meets tol."""
    et = op.prepare_source(scheme, eta)
    mask, fill = op.solve_subspace(scheme)
    if mask is None:
        A = lambda v: op.prec(scheme, v)
        Ad = lambda v: op.prec_dag(scheme, v)
        rhs = et
    else:
        A = lambda v: mask * op.prec(scheme, mask * v)
        Ad = lambda v: mask * op.prec_dag(scheme, mask * v)
        rhs = mask * et
    etan = np.sqrt(_nrm2(eta))
    inner_tol = 0.5 * tol * etan / np.sqrt(_nrm2(rhs))
    y = None
    total = 0
    for _ in range(5):
        if solver == "cgnr":
            y, info = cgnr(A, Ad, rhs, inner_tol, maxiter, y)
        else:
            y, info = bicgstab(A, rhs, inner_tol, maxiter, y)
        total += info["iters"]
        yfull = y if mask is None else y + fill(et)
        x = op.reconstruct(scheme, yfull)
        true = np.sqrt(_nrm2(eta - op.M(x))) / etan
        if true <= tol:
            break
        inner_tol *= 0.1
    info = dict(info)
    info.update(iters=total, true_rel_resid=true)
    return x, info
