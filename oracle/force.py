"""Gradient of L = |x|^2, x = M^-1 eta, with respect to the links and the source.

Conventions (PyTorch's for complex tensors): for real L, grad_z is the tensor with
dL = Re <grad_z, dz> summed over components.  Then
    g = 2 x,   M^dagger lambda = g,   grad_eta = lambda.
`link_gradient` differentiates the hopping terms (the SW term A held fixed);
`clover_gradient` adds the derivative of A(U) through the four-leaf field strength;
their sum is the whole link gradient.

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


def _torch_clover(U, c_s, c_t):
    """A(U) of wilson.clover_field written with torch CPU ops, so that it can be
    differentiated: -(c/2) sum_planes sigma_{mu nu} (x) F_{mu nu}, F the traceless
    anti-hermitian part of the four-leaf sum Q / 8 (leaves oriented mu -> nu)."""
    import torch

    from .dirac import sigma

    dag = lambda m: m.conj().transpose(-1, -2)
    sh = lambda f, d, k: torch.roll(f, shifts=-k, dims=AXIS[d])
    site_shape = U.shape[1:5]
    A = torch.zeros(site_shape + (12, 12), dtype=torch.complex128)
    planes = [(0, 3, c_t), (1, 3, c_t), (2, 3, c_t), (0, 1, c_s), (0, 2, c_s), (1, 2, c_s)]
    for mu, nu, c in planes:
        if c == 0.0:
            continue
        um, un = U[mu], U[nu]
        l1 = um @ sh(un, mu, 1) @ dag(sh(um, nu, 1)) @ dag(un)
        l2 = un @ dag(sh(sh(um, mu, -1), nu, 1)) @ dag(sh(un, mu, -1)) @ sh(um, mu, -1)
        l3 = dag(sh(um, mu, -1)) @ dag(sh(sh(un, mu, -1), nu, -1)) @ sh(sh(um, mu, -1), nu, -1) @ sh(un, nu, -1)
        l4 = dag(sh(un, nu, -1)) @ sh(um, nu, -1) @ sh(sh(un, mu, 1), nu, -1) @ dag(um)
        q = l1 + l2 + l3 + l4
        f = (q - dag(q)) / 8.0
        tr = torch.diagonal(f, dim1=-2, dim2=-1).sum(-1) / 3.0
        f = f - tr[..., None, None] * torch.eye(3, dtype=torch.complex128)
        s = torch.from_numpy(sigma(mu, nu))
        A = A + (-(c / 2.0)) * torch.einsum("st,...ab->...satb", s, f).reshape(site_shape + (12, 12))
    return A


def clover_gradient(op, x, lam):
    """(grad_U, G) of the SW term's dependence on the links: dL = -Re <lambda, dA x>.
    The raw gradient is that of s(U) = -Re sum_x lambda(x)^dagger A(U)(x) x(x) by reverse-mode
    differentiation (torch), with dL = Re <grad_U, dU>; G is its su(3) projection as in
    link_gradient."""
    import torch

    Ut = torch.from_numpy(np.ascontiguousarray(op.U)).clone().requires_grad_(True)
    A = _torch_clover(Ut, op.c_s, op.c_t)
    xs = torch.from_numpy(np.ascontiguousarray(x)).reshape(x.shape[:4] + (12,))
    ls = torch.from_numpy(np.ascontiguousarray(lam)).reshape(lam.shape[:4] + (12,))
    s = -torch.einsum("...i,...ij,...j->", ls.conj(), A, xs).real
    (g,) = torch.autograd.grad(s, Ut)
    grad = g.numpy()
    iug = 1j * (op.U @ _dag(grad))
    h = (iug + _dag(iug)) / 2
    tr = np.trace(h, axis1=-2, axis2=-1) / 3.0
    G = h - tr[..., None, None] * np.eye(3)
    return grad, G


def full_link_gradient(op, x, lam):
    """Hopping plus SW-term link gradient: the whole dL/dU of L with A = A(U)."""
    g, G = link_gradient(op, x, lam)
    if op.clover:
        gc, Gc = clover_gradient(op, x, lam)
        g, G = g + gc, G + Gc
    return g, G
