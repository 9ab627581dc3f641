"""Gradient of L = |x|^2, x = M^-1 eta, with respect to the links and the source.

Conventions (PyTorch's for complex tensors): for real L, grad_z is the tensor with
dL = Re <grad_z, dz> summed over components.  Then
    g = 2 x,   M^dagger lambda = g,   grad_eta = lambda.
Only the hopping terms are differentiated: the SW term A is held fixed, so the
link gradient is the full one when c_s = c_t = 0.

With kappa_t = 1, kappa_i = 1/gamma_f and b_mu(s) = b on the time links of the
last time slice (1 elsewhere), the hop contributes, per link U_mu(s),
    Y = sum_alpha [P-^mu x(s+mu)]_alpha lambda(s)_alpha^dagger,
    Z = sum_alpha [P+^mu x(s)]_alpha lambda(s+mu)_alpha^dagger,
    grad_U = kappa_mu b_mu(s) (Y + Z^dagger)^dagger,
and for a link moved along U -> exp(i h omega) U, omega hermitian traceless,
    dL/dh = tr(omega G),   G = kappa_mu b_mu(s) TH[i U (Y + Z^dagger)],
with TH(K) = (K + K^dagger)/2 - tr(K + K^dagger)/6 (the su(3) projection).
"""
import numpy as np

from .dirac import P_MINUS, P_PLUS, spin_apply
from .wilson import AXIS
from .krylov import solve


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def link_gradient(op, x, lam):
    """(grad_U [4,...,3,3], G [4,...,3,3]) from x and lambda = M^-dagger (2x)."""
    U = op.U
    nt = U.shape[1]
    grad = np.zeros_like(U)
    G = np.zeros_like(U)
    for mu in range(4):
        ax = AXIS[mu]
        kappa = 1.0 if mu == 3 else 1.0 / op.gamma_f
        xf = np.roll(x, -1, axis=ax)
        lf = np.roll(lam, -1, axis=ax)
        Y = np.einsum("...sc,...sa->...ca", spin_apply(P_MINUS[mu], xf), lam.conj())
        Z = np.einsum("...sc,...sa->...ca", spin_apply(P_PLUS[mu], x), lf.conj())
        K = Y + _dag(Z)
        fac = np.full(U.shape[1:5], kappa)
        if mu == 3:
            fac[nt - 1] *= op.b
        grad[mu] = fac[..., None, None] * _dag(K)
        iuk = 1j * (U[mu] @ K)
        h = (iuk + _dag(iuk)) / 2
        tr = np.trace(h, axis1=-2, axis2=-1) / 3.0
        G[mu] = fac[..., None, None] * (h - tr[..., None, None] * np.eye(3))
    return grad, G


def loss_and_grads(op, eta, scheme="TEMPORAL_SCHUR", tol=1e-13):
    """L, grad_eta, grad_U, G for L = |M^-1 eta|^2, solving both systems tightly."""
    x, _ = solve(op, scheme, eta, "bicgstab", tol)
    g = 2.0 * x
    # M^dagger lambda = g  <=>  M (gamma5 lambda) = gamma5 g
    from .dirac import GAMMA5
    y, _ = solve(op, scheme, spin_apply(GAMMA5, g), "bicgstab", tol)
    lam = spin_apply(GAMMA5, y)
    grad_U, G = link_gradient(op, x, lam)
    return float(np.vdot(x, x).real), lam, grad_U, G, x
