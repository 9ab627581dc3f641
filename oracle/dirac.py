"""Spin matrices in the Dirac-Pauli basis (gamma_t diagonal, Appendix C).

Direction index 0=x, 1=y, 2=z, 3=t.  The paper writes the temporal matrix as
gamma_0; here it is ``GAMMA[3]``.

    gamma_t = diag(1, 1, -1, -1)
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]      k = x, y, z
    gamma_5 = gamma_x gamma_y gamma_z gamma_t

All four are hermitian and obey {gamma_mu, gamma_nu} = 2 delta_{mu nu}.
Projectors P+-^mu = (1 +- gamma_mu)/2 (Sec. II, definition of D_t and D_s), and
sigma_{mu nu} = [gamma_mu, gamma_nu] / 2 (Sec. II, the SW term).
"""
import numpy as np

_pauli = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
_z2 = np.zeros((2, 2), dtype=np.complex128)

GAMMA = np.zeros((4, 4, 4), dtype=np.complex128)
for _k in range(3):
    GAMMA[_k] = np.block([[_z2, -1j * _pauli[_k]], [1j * _pauli[_k], _z2]])
GAMMA[3] = np.diag([1, 1, -1, -1]).astype(np.complex128)

GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

ID4 = np.eye(4, dtype=np.complex128)

# P_minus[mu] = (1 - gamma_mu)/2 multiplies the forward hop, P_plus the backward hop.
P_MINUS = np.array([(ID4 - GAMMA[m]) / 2 for m in range(4)])
P_PLUS = np.array([(ID4 + GAMMA[m]) / 2 for m in range(4)])

# Temporal projectors of Sec. II.A: P+- = (1 +- gamma_t)/2.
PT_PLUS = P_PLUS[3]
PT_MINUS = P_MINUS[3]


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = [gamma_mu, gamma_nu]/2 (anti-hermitian)."""
    return (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu]) / 2


def spin_apply(s: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to a field [..., 4, 3]."""
    return np.einsum("st,...tc->...sc", s, psi)


def g5(psi: np.ndarray) -> np.ndarray:
    return spin_apply(GAMMA5, psi)
