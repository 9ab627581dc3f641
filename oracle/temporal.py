"""The temporal preconditioner (Sec. II.A).

Per spatial site the temporal matrix acts on colour vectors along the time line,
    (T psi)(t) = mu psi(t) - U_t(t) psi(t+1),
where the wrap t = Nt-1 -> 0 carries the fermion boundary phase b, i.e. the
corner entry is T_{Nt-1,0} = -b U_t(Nt-1).  (This is the reading under which
mu - D_t = C_L^-1 C_R^-1 holds with D_t's own boundary phase; the printed
eq:boundary transposes the corner and flips the sign.)

T^-1 is applied with the Sherman-Morrison-Woodbury split T = T0 + V W^dagger of
eq:SMW1: T0 is T without the corner (upper bidiagonal), V carries the corner in
the last time slice, W selects time slice 0.  The set-up computes X = T0^-1 V by
back-substitution and Lambda = (I + W^dagger X)^-1 = (I + X(0))^-1; an apply
back-substitutes chi = T0^-1 eta, forms q = Lambda chi(0) and returns
psi = chi - X q.  Back-substitution reads chi(t) = (eta(t) + U_t(t) chi(t+1))/mu,
the sign that follows from T's definition (the appendix's FLOP-count step prints
a minus, which does not change the count).

T^dagger^-1 uses the mirrored split (Sec. II.A, closing paragraphs): forward
substitution from t=0, V' = -b U_t(Nt-1)^dagger in time slice 0 and W' selecting
time slice Nt-1, so X'(Nt-1) builds up to the adjoint Polyakov loop.

C_L = P+ + P- T^-1 and C_R = P- + P+ T^dagger^-1 with P+- = (1 +- gamma_t)/2.

The cutoff trick (Sec. II.A, eq:cutoff): X(t) is a product of unitary time links divided by
mu^(Nt-t), so ||X(t)||_F = sqrt(3) mu^-(Nt-t); where that bound is below a threshold eps the
correction X(t) q is dropped (X(t) set to zero).  For T^dagger the suppression runs the other
way, ||X'(t)||_F = sqrt(3) mu^-(t+1).  eps = 0 keeps the exact inverse.
"""
import numpy as np

from .dirac import PT_PLUS, PT_MINUS, spin_apply
from .wilson import colour_apply, colour_apply_dag, shift, link_shift


def _matvec(m, v):
    """m [...,3,3] times v [...,4,3] (each spin)."""
    return np.einsum("...ab,...sb->...sa", m, v)


def apply_T(Ut, psi, mu, b=-1.0):
    return mu * psi - colour_apply(Ut, shift(psi, 3, +1, b))


def apply_Tdag(Ut, psi, mu, b=-1.0):
    return mu * psi - colour_apply_dag(link_shift(Ut, 3, -1), shift(psi, 3, -1, b))


def smw_setup(Ut, mu, b=-1.0):
    """X = T0^-1 V by back-substitution, and Lambda = (I + X(0))^-1.

    Returns X [Lt,Lz,Ly,Lx,3,3] and Lambda [Lz,Ly,Lx,3,3]."""
    nt = Ut.shape[0]
    X = np.empty_like(Ut)
    X[nt - 1] = -b * Ut[nt - 1] / mu
    for t in range(nt - 2, -1, -1):
        X[t] = Ut[t] @ X[t + 1] / mu
    lam = np.linalg.inv(np.eye(3) + X[0])
    return X, lam


def smw_setup_dag(Ut, mu, b=-1.0):
    """Mirror set-up for T^dagger: X'(0) = -b U(Nt-1)^dagger/mu, X'(t) = U(t-1)^dagger X'(t-1)/mu."""
    nt = Ut.shape[0]
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    X = np.empty_like(Ut)
    X[0] = -b * dag(Ut[nt - 1]) / mu
    for t in range(1, nt):
        X[t] = dag(Ut[t - 1]) @ X[t - 1] / mu
    lam = np.linalg.inv(np.eye(3) + X[nt - 1])
    return X, lam


def cutoff_slices(nt, mu, eps, dagger=False):
    """Time slices whose Woodbury vector the cutoff trick drops: where the eq:cutoff bound
    sqrt(3) mu^-(Nt-t) (T^-1) or sqrt(3) mu^-(t+1) (T^dagger^-1) is below eps."""
    t = np.arange(nt)
    bound = np.sqrt(3.0) * float(mu) ** -((t + 1) if dagger else (nt - t)).astype(np.float64)
    return bound < eps


def apply_Tinv(Ut, eta, mu, b=-1.0, setup=None, eps=0.0):
    """psi = T^-1 eta on every spin component of eta [Lt,Lz,Ly,Lx,4,3]; with eps > 0 the
    cutoff trick zeroes X(t) where its norm bound is below eps."""
    X, lam = setup if setup is not None else smw_setup(Ut, mu, b)
    nt = Ut.shape[0]
    chi = np.empty_like(eta)
    chi[nt - 1] = eta[nt - 1] / mu
    for t in range(nt - 2, -1, -1):
        chi[t] = (eta[t] + _matvec(Ut[t], chi[t + 1])) / mu
    q = _matvec(lam, chi[0])
    drop = cutoff_slices(nt, mu, eps)
    return chi - np.stack([np.zeros_like(chi[t]) if drop[t] else _matvec(X[t], q) for t in range(nt)])


def apply_Tdaginv(Ut, eta, mu, b=-1.0, setup=None, eps=0.0):
    """psi = (T^dagger)^-1 eta by forward substitution plus the mirrored Woodbury step (with
    the mirrored cutoff trick for eps > 0)."""
    X, lam = setup if setup is not None else smw_setup_dag(Ut, mu, b)
    nt = Ut.shape[0]
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    chi = np.empty_like(eta)
    chi[0] = eta[0] / mu
    for t in range(1, nt):
        chi[t] = (eta[t] + _matvec(dag(Ut[t - 1]), chi[t - 1])) / mu
    q = _matvec(lam, chi[nt - 1])
    drop = cutoff_slices(nt, mu, eps, dagger=True)
    return chi - np.stack([np.zeros_like(chi[t]) if drop[t] else _matvec(X[t], q) for t in range(nt)])


class Temporal:
    """C_L, C_R and their inverses for one gauge field and mass (Sec. II.A); eps > 0 applies
    the cutoff trick in T^-1 and T^dagger^-1 (so C_L, C_R are then approximate inverses)."""

    def __init__(self, U, mu, b=-1.0, eps=0.0):
        self.Ut = U[3]
        self.mu = mu
        self.b = b
        self.eps = eps
        self.fwd = smw_setup(self.Ut, mu, b)
        self.bwd = smw_setup_dag(self.Ut, mu, b)

    def Tinv(self, psi):
        return apply_Tinv(self.Ut, psi, self.mu, self.b, self.fwd, self.eps)

    def Tdaginv(self, psi):
        return apply_Tdaginv(self.Ut, psi, self.mu, self.b, self.bwd, self.eps)

    def T(self, psi):
        return apply_T(self.Ut, psi, self.mu, self.b)

    def Tdag(self, psi):
        return apply_Tdag(self.Ut, psi, self.mu, self.b)

    def CL(self, psi):
        """C_L = P+ + P- T^-1."""
        return spin_apply(PT_PLUS, psi) + spin_apply(PT_MINUS, self.Tinv(psi))

    def CR(self, psi):
        """C_R = P- + P+ (T^dagger)^-1."""
        return spin_apply(PT_MINUS, psi) + spin_apply(PT_PLUS, self.Tdaginv(psi))

    def CL_inv(self, psi):
        """C_L^-1 = P+ + P- T."""
        return spin_apply(PT_PLUS, psi) + spin_apply(PT_MINUS, self.T(psi))

    def CR_inv(self, psi):
        """C_R^-1 = P- + P+ T^dagger."""
        return spin_apply(PT_MINUS, psi) + spin_apply(PT_PLUS, self.Tdag(psi))
