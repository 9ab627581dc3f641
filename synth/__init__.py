"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and shapes them into lattice fields.  It
contains none of the arithmetic of the preconditioned Wilson/clover method: no
hopping terms, no temporal inverses, no Krylov steps.  Both the FP64 oracle
(``oracle/``) and the HIP library's callers take their inputs from here so that
the two sides see bit-identical data.

Canonical layouts (complex128, C order):
    links   : [4][Lt][Lz][Ly][Lx][3][3]   direction index 0=x, 1=y, 2=z, 3=t
    spinor  : [Lt][Lz][Ly][Lx][4][3]      spin (Dirac-Pauli basis) then colour
    gauge transform : [Lt][Lz][Ly][Lx][3][3]

The paper's workloads are quenched Wilson-gauge ensembles (Sec. III, Table I),
which are not available here.  Links are instead U = exp(i eps_mu H) with H a
Gaussian traceless hermitian 3x3 matrix, with separate eps for spatial and
temporal links, which gives SU(3) fields whose plaquette can be tuned towards
the paper's u_s range.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "su3_algebra",
    "make_links",
    "make_source",
    "make_point_source",
    "make_gauge_transform",
    "make_algebra_field",
    "unit_links",
    "abelian_plane_links",
    "WORKLOADS",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), normalised tr(l_a l_b) = 2 delta_ab."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j
    l[1, 1, 0] = 1j
    l[2, 0, 0] = 1
    l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j
    l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j
    l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def su3_algebra(omega: np.ndarray) -> np.ndarray:
    """Hermitian traceless H = sum_a omega_a lambda_a / 2 from coefficients [..., 8]."""
    return np.einsum("...a,aij->...ij", omega, gell_mann()) * 0.5


def _expi(h: np.ndarray, eps) -> np.ndarray:
    """exp(i eps h) for hermitian h [..., 3, 3] via its eigendecomposition."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * np.asarray(eps)[..., None] * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def make_links(dims, eps_s: float, eps_t: float, seed: int) -> np.ndarray:
    """SU(3) links U_mu(x) = exp(i eps_mu H_mu(x)), canonical [4][Lt][Lz][Ly][Lx][3][3].

    dims = (Lx, Ly, Lz, Lt).  The eight algebra coefficients of every link are
    drawn in one call of numpy's PCG64 generator, shape (4, Lt, Lz, Ly, Lx, 8).
    """
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((4, lt, lz, ly, lx, 8))
    h = su3_algebra(omega)
    eps = np.empty((4, lt, lz, ly, lx))
    eps[:3] = eps_s
    eps[3] = eps_t
    return np.ascontiguousarray(_expi(h, eps))


def unit_links(dims) -> np.ndarray:
    """Free field: every link is the identity."""
    lx, ly, lz, lt = dims
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def abelian_plane_links(dims, mu: int, nu: int, n: int = 1) -> np.ndarray:
    """Constant abelian field in the (mu, nu) plane.

    U_mu(x) = exp(-i f x_nu D), D = diag(1, -1, 0), f = 2 pi n / L_nu; every other
    link is the identity.  Every plaquette of the (mu, nu) plane then equals
    exp(i f D) exactly, for any position, including across the periodic wrap.
    """
    u = unit_links(dims)
    lnu = dims[nu]
    f = 2 * np.pi * n / lnu
    shape_axes = {0: 3, 1: 2, 2: 1, 3: 0}  # direction -> axis of [Lt][Lz][Ly][Lx]
    coord = np.arange(lnu)
    bshape = [1, 1, 1, 1]
    bshape[shape_axes[nu]] = lnu
    xnu = coord.reshape(bshape)
    ph1 = np.exp(-1j * f * xnu)
    ph2 = np.exp(+1j * f * xnu)
    full = np.broadcast_to(ph1, u.shape[1:5])
    u[mu, ..., 0, 0] = full
    u[mu, ..., 1, 1] = np.broadcast_to(ph2, u.shape[1:5])
    u[mu, ..., 2, 2] = 1
    return u


def make_source(dims, seed: int) -> np.ndarray:
    """Gaussian complex spinor: Re and Im iid N(0,1), canonical [Lt][Lz][Ly][Lx][4][3]."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((lt, lz, ly, lx, 4, 3, 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def make_point_source(dims, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """Unit spin-colour vector at one site (x, y, z, t)."""
    lx, ly, lz, lt = dims
    e = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    x, y, z, t = site
    e[t, z, y, x, spin, colour] = 1
    return e


def make_gauge_transform(dims, seed: int) -> np.ndarray:
    """Haar-random SU(3) matrix per site, canonical [Lt][Lz][Ly][Lx][3][3].

    QR of a complex Gaussian matrix with the phases of R's diagonal moved into Q
    (Mezzadri's recipe), then the determinant phase divided out.
    """
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((lt, lz, ly, lx, 3, 3, 2))
    a = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2)
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[..., None, None]
    return np.ascontiguousarray(q)


def make_algebra_field(dims, seed: int) -> np.ndarray:
    """Random su(3) direction per link: hermitian traceless [4][Lt][Lz][Ly][Lx][3][3]."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((4, lt, lz, ly, lx, 8))
    return np.ascontiguousarray(su3_algebra(omega))


# Workload presets.  gamma_f = xi (bare anisotropy, nu = 1); m0 = -0.05 for all;
# c_s = csw_s / gamma_f, c_t = csw_t; antiperiodic time (b = -1).
WORKLOADS = {
    "wilson_4x16": dict(dims=(4, 4, 4, 16), xi=3.0, m0=-0.05, csw_s=0.0, csw_t=0.0,
                        eps_s=0.3, eps_t=0.1, seed=1000),
    "clover_16x128": dict(dims=(16, 16, 16, 128), xi=3.5, m0=-0.05, csw_s=1.6, csw_t=1.0,
                          eps_s=0.35, eps_t=0.12, seed=1001),
    "clover_24x128": dict(dims=(24, 24, 24, 128), xi=5.0, m0=-0.05, csw_s=1.6, csw_t=1.0,
                          eps_s=0.35, eps_t=0.12, seed=1002),
    "clover_12x64": dict(dims=(12, 12, 12, 64), xi=3.0, m0=-0.05, csw_s=1.6, csw_t=1.0,
                         eps_s=0.35, eps_t=0.12, seed=1003),
    "clover_32x256": dict(dims=(32, 32, 32, 256), xi=6.0, m0=-0.05, csw_s=1.6, csw_t=1.0,
                          eps_s=0.4, eps_t=0.1, seed=1004),
    "clover_32x32_iso": dict(dims=(32, 32, 32, 32), xi=1.0, m0=-0.05, csw_s=1.6, csw_t=1.0,
                             eps_s=0.4, eps_t=0.1, seed=1050),
}
