"""The anisotropic Wilson / SW fermion matrix (Sec. II, opening definitions).

    M = A + mu - D_t - D_s / gamma_f,      mu = m0 + 1 + 3 / gamma_f
    D_mu psi(x) = P-^mu U_mu(x) psi(x + mu) + P+^mu U_mu(x - mu)^dagger psi(x - mu)
    D_s = D_x + D_y + D_z,  D_t = D_(direction 3)

Lattice units with a_t = 1, so the paper's a_t m0 is m0.  Space is periodic; a hop
across the time boundary picks up the phase b (+1 periodic, -1 antiperiodic).

The SW term (same section) is the site-diagonal hermitian 12x12 matrix
    A = -(c_t/2) sum_i sigma_{i t} F_{i t} - (c_s/2) sum_{i<j} sigma_{ij} F_{ij}
with F_{mu nu} the anti-hermitian traceless clover-leaf field strength
    F = (Q - Q^dagger)/8 - trace/3,  Q = sum of the four plaquette leaves at x,
all oriented mu -> nu.  Each spatial plane is counted once (i<j), so that the
isotropic case c_s = c_t weights every plane equally.
"""
import numpy as np

from .dirac import P_MINUS, P_PLUS, sigma, spin_apply, GAMMA5

# direction -> axis of a site-shaped array [Lt][Lz][Ly][Lx]
AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def mass_term(m0: float, gamma_f: float) -> float:
    """mu = m0 + 1 + 3/gamma_f (a_t = 1)."""
    return m0 + 1.0 + 3.0 / gamma_f


def shift(psi: np.ndarray, mu: int, sign: int, b: float = 1.0) -> np.ndarray:
    """Return psi(x + sign*mu_hat) for a field whose first four axes are sites.

    Across the time boundary the value is multiplied by b (fermion BC)."""
    ax = AXIS[mu]
    out = np.roll(psi, -sign, axis=ax)
    if mu == 3 and b != 1.0:
        out = out.copy()
        if sign > 0:
            out[-1] *= b
        else:
            out[0] *= b
    return out


def link_shift(u_mu: np.ndarray, mu_dir: int, sign: int) -> np.ndarray:
    """A link field [Lt][Lz][Ly][Lx][3][3] evaluated at x + sign*dir (periodic)."""
    return np.roll(u_mu, -sign, axis=AXIS[mu_dir])


def colour_apply(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """u(x) v(x) for u [...,3,3] and v [...,4,3] (all spins)."""
    return np.einsum("...ab,...sb->...sa", u, v)


def colour_apply_dag(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """u(x)^dagger v(x)."""
    return np.einsum("...ba,...sb->...sa", u.conj(), v)


def hop(U: np.ndarray, psi: np.ndarray, mu: int, b: float = 1.0) -> np.ndarray:
    """D_mu psi, the forward and backward hop in direction mu."""
    fwd = colour_apply(U[mu], shift(psi, mu, +1, b))
    bwd = colour_apply_dag(link_shift(U[mu], mu, -1), shift(psi, mu, -1, b))
    return spin_apply(P_MINUS[mu], fwd) + spin_apply(P_PLUS[mu], bwd)


def hop_s(U, psi, b=1.0):
    """D_s = sum over the three spatial directions."""
    return hop(U, psi, 0, b) + hop(U, psi, 1, b) + hop(U, psi, 2, b)


def hop_t(U, psi, b=1.0):
    return hop(U, psi, 3, b)


def apply_A(A: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Site-diagonal 12x12 matrix [..., 12, 12] (index spin*3+colour) times psi [..., 4, 3]."""
    sh = psi.shape
    v = psi.reshape(sh[:-2] + (12,))
    return np.einsum("...ij,...j->...i", A, v).reshape(sh)


def apply_M(U, psi, m0, gamma_f, b=-1.0, A=None):
    """M psi = A psi + mu psi - D_t psi - D_s psi / gamma_f."""
    mu = mass_term(m0, gamma_f)
    out = mu * psi - hop_t(U, psi, b) - hop_s(U, psi, b) / gamma_f
    if A is not None:
        out = out + apply_A(A, psi)
    return out


def apply_Mdag(U, psi, m0, gamma_f, b=-1.0, A=None):
    """M^dagger = gamma5 M gamma5 (the hopping terms and A are gamma5-hermitian)."""
    return spin_apply(GAMMA5, apply_M(U, spin_apply(GAMMA5, psi), m0, gamma_f, b, A))


def plaquette_leaves(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): the sum of the four plaquettes at x, each oriented mu -> nu."""
    um, un = U[mu], U[nu]
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    mm = lambda *ms: _chain(ms)
    sm = lambda f, d, s: link_shift(f, d, s)
    # leaf 1: +mu, +nu, -mu, -nu
    l1 = mm(um, sm(un, mu, +1), dag(sm(um, nu, +1)), dag(un))
    # leaf 2: +nu, -mu, -nu, +mu
    u_m_pn = sm(sm(um, mu, -1), nu, +1)      # U_mu(x - mu + nu)
    l2 = mm(un, dag(u_m_pn), dag(sm(un, mu, -1)), sm(um, mu, -1))
    # leaf 3: -mu, -nu, +mu, +nu
    u_m_mn = sm(sm(um, mu, -1), nu, -1)      # U_mu(x - mu - nu)
    u_n_mn = sm(sm(un, mu, -1), nu, -1)      # U_nu(x - mu - nu)
    l3 = mm(dag(sm(um, mu, -1)), dag(u_n_mn), u_m_mn, sm(un, nu, -1))
    # leaf 4: -nu, +mu, +nu, -mu
    u_n_pm_mn = sm(sm(un, mu, +1), nu, -1)   # U_nu(x + mu - nu)
    l4 = mm(dag(sm(un, nu, -1)), sm(um, nu, -1), u_n_pm_mn, dag(um))
    return l1 + l2 + l3 + l4


def _chain(ms):
    out = ms[0]
    for m in ms[1:]:
        out = out @ m
    return out


def field_strength(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Anti-hermitian traceless F_{mu nu} = (Q - Q^dagger)/8 - tr/3."""
    q = plaquette_leaves(U, mu, nu)
    f = (q - np.conj(np.swapaxes(q, -1, -2))) / 8.0
    tr = np.trace(f, axis1=-2, axis2=-1) / 3.0
    return f - tr[..., None, None] * np.eye(3)


def clover_field(U: np.ndarray, c_s: float, c_t: float) -> np.ndarray:
    """The SW term A(x) as a 12x12 matrix per site, index spin*3 + colour.

    A = -(c_t/2) sum_i sigma_{it} F_{it} - (c_s/2) sum_{i<j} sigma_{ij} F_{ij}.
    Built from the raw (periodic) links; a time-boundary phase b cancels in
    every closed loop.
    """
    site_shape = U.shape[1:5]
    A = np.zeros(site_shape + (12, 12), dtype=np.complex128)
    planes = [(0, 3, c_t), (1, 3, c_t), (2, 3, c_t), (0, 1, c_s), (0, 2, c_s), (1, 2, c_s)]
    for mu, nu, c in planes:
        if c == 0.0:
            continue
        f = field_strength(U, mu, nu)
        s = sigma(mu, nu)
        A += -(c / 2.0) * np.einsum("st,...ab->...satb", s, f).reshape(site_shape + (12, 12))
    return A


def clover_plus_mass_inverse(A: np.ndarray, mu: float) -> np.ndarray:
    """(A + mu)^-1 per site by a dense 12x12 inverse."""
    return np.linalg.inv(A + mu * np.eye(12))
