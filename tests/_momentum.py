"""Free-field (U = 1) momentum-space closed forms used to pin the oracle.

A plane wave psi(x) = exp(i p.x) u is an eigenvector of every hop:
    D_mu psi = (cos p_mu - i gamma_mu sin p_mu) psi,
so the fermion matrix of Sec. II becomes the 4x4 matrix
    M(p) = W(p) + i (gamma_t sin p_t + sum_k gamma_k sin p_k / gamma_f),
    W(p) = m0 + (1 - cos p_t) + sum_k (1 - cos p_k) / gamma_f,
with p_k = 2 pi n_k / L_k and p_t = 2 pi (n + 1/2) / Lt for an antiperiodic time
direction.  Its singular values are sqrt(W^2 + s^2), s^2 = sin^2 p_t +
sum_k sin^2 p_k / gamma_f^2.  The temporal matrix is T(p) = mu - exp(i p_t).

Written independently of ``oracle/`` (no shared code) from these formulas.
"""
import numpy as np

_s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
      np.array([[1, 0], [0, -1]], complex)]
_z = np.zeros((2, 2), complex)
G = [np.block([[_z, -1j * s], [1j * s, _z]]) for s in _s] + [np.diag([1, 1, -1, -1]).astype(complex)]
I4 = np.eye(4, dtype=complex)


def momenta(dims, b):
    """Arrays of allowed (px, py, pz, pt) for periodic space and time phase b."""
    lx, ly, lz, lt = dims
    shift = 0.5 if b < 0 else 0.0
    px = 2 * np.pi * np.arange(lx) / lx
    py = 2 * np.pi * np.arange(ly) / ly
    pz = 2 * np.pi * np.arange(lz) / lz
    pt = 2 * np.pi * (np.arange(lt) + shift) / lt
    return px, py, pz, pt


def apply_M_fft(psi, m0, gamma_f, b):
    """Free-field M psi evaluated in momentum space (canonical [Lt,Lz,Ly,Lx,4,3])."""
    lt, lz, ly, lx = psi.shape[:4]
    px, py, pz, pt = momenta((lx, ly, lz, lt), b)
    t = np.arange(lt).reshape(lt, 1, 1, 1, 1, 1)
    twist = np.exp(1j * np.pi * t / lt) if b < 0 else 1.0
    f = np.fft.fftn(psi / twist, axes=(0, 1, 2, 3))
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    W = m0 + (1 - np.cos(PT)) + ((1 - np.cos(PX)) + (1 - np.cos(PY)) + (1 - np.cos(PZ))) / gamma_f
    Mp = (W[..., None, None] * I4
          + 1j * (np.sin(PT)[..., None, None] * G[3]
                  + (np.sin(PX)[..., None, None] * G[0] + np.sin(PY)[..., None, None] * G[1]
                     + np.sin(PZ)[..., None, None] * G[2]) / gamma_f))
    g = np.einsum("...st,...tc->...sc", Mp, f)
    return np.fft.ifftn(g, axes=(0, 1, 2, 3)) * twist


def singular_values(dims, m0, gamma_f, b):
    px, py, pz, pt = momenta(dims, b)
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    W = m0 + (1 - np.cos(PT)) + ((1 - np.cos(PX)) + (1 - np.cos(PY)) + (1 - np.cos(PZ))) / gamma_f
    s2 = np.sin(PT) ** 2 + (np.sin(PX) ** 2 + np.sin(PY) ** 2 + np.sin(PZ) ** 2) / gamma_f ** 2
    return np.sqrt(W ** 2 + s2).ravel()


def _blocks(dims, m0, gamma_f, b):
    px, py, pz, pt = momenta(dims, b)
    PT, PZ, PY, PX = [a.ravel() for a in np.meshgrid(pt, pz, py, px, indexing="ij")]
    mu = m0 + 1 + 3 / gamma_f
    n = PT.size
    Ds = np.zeros((n, 4, 4), complex)
    for k, P in enumerate((PX, PY, PZ)):
        Ds += np.cos(P)[:, None, None] * I4 - 1j * np.sin(P)[:, None, None] * G[k]
    Dt = np.cos(PT)[:, None, None] * I4 - 1j * np.sin(PT)[:, None, None] * G[3]
    Pp, Pm = (I4 + G[3]) / 2, (I4 - G[3]) / 2
    Tinv = 1.0 / (mu - np.exp(1j * PT))
    Tdinv = 1.0 / (mu - np.exp(-1j * PT))
    CL = Pp[None] + Pm[None] * Tinv[:, None, None]
    CR = Pm[None] + Pp[None] * Tdinv[:, None, None]
    return mu, Ds, Dt, CL, CR


def kappa_free(dims, m0, gamma_f, b, scheme):
    """kappa(Mt^dagger Mt) of each scheme's free-field operator from 4x4 blocks.

    UNPREC: M(p).  SCHUR4D: mu - D_w(p)^2/mu (D_w(p+pi) = -D_w(p) keeps the odd
    block diagonal in p).  TEMPORAL: 1 - C_L D_s C_R/gamma_f.  TEMPORAL_SCHUR
    (Wilson): 1 - (C_L D_s C_R)^2/gamma_f^2, since D_s(p + pi_s) = -D_s(p) and
    C_L, C_R do not depend on the spatial momentum.  TEMPORAL_SCHUR3D: C_L S_o C_R with the
    Schur complement S_o = mu - D_t - D_s (mu - D_t)^-1 D_s/gamma_f^2 taken as defined.
    TEMPORAL_FULLSW: 1 - (mu - D_t)^-1 D_s/gamma_f (T = mu - D_t for the free Wilson field)."""
    mu, Ds, Dt, CL, CR = _blocks(dims, m0, gamma_f, b)
    if scheme == "UNPREC":
        m = mu * I4 - Dt - Ds / gamma_f
    elif scheme == "SCHUR4D":
        Dw = Dt + Ds / gamma_f
        m = mu * I4 - Dw @ Dw / mu
    elif scheme == "TEMPORAL":
        m = I4 - CL @ Ds @ CR / gamma_f
    elif scheme == "TEMPORAL_SCHUR":
        db = CL @ Ds @ CR
        m = I4 - db @ db / gamma_f ** 2
    elif scheme == "TEMPORAL_SCHUR3D":
        mee = mu * I4 - Dt
        m = CL @ (mee - Ds @ np.linalg.inv(mee) @ Ds / gamma_f ** 2) @ CR
    elif scheme == "TEMPORAL_FULLSW":
        m = I4 - np.linalg.inv(mu * I4 - Dt) @ Ds / gamma_f
    else:
        raise ValueError(scheme)
    sv = np.linalg.svd(m, compute_uv=False)
    return (sv.max() / sv.min()) ** 2
