"""Pins of the oracle's fermion matrix and SW term (Sec. II) against mathematics
that does not come from the oracle itself."""
import numpy as np
import pytest

import synth
from oracle import dirac, wilson as W
from oracle.schemes import Operator
import _momentum as mom


def test_gamma_clifford_and_basis():
    g = dirac.GAMMA
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * (m == n) * np.eye(4))
    # Dirac-Pauli basis: gamma_t diagonal, so P+ keeps the upper two spins.
    assert np.allclose(dirac.PT_PLUS, np.diag([1, 1, 0, 0]))
    g5 = dirac.GAMMA5
    assert np.allclose(g5 @ g5, np.eye(4))
    for m in range(4):
        assert np.allclose(g5 @ g[m], -g[m] @ g5)
    # gamma5 swaps upper and lower spin pairs with a minus sign in this basis
    assert np.allclose(g5, np.block([[np.zeros((2, 2)), -np.eye(2)], [-np.eye(2), np.zeros((2, 2))]]))


@pytest.mark.parametrize("dims,m0,gf,b", [((4, 4, 4, 8), -0.05, 3.0, -1.0),
                                         ((2, 4, 6, 4), 0.3, 1.0, -1.0),
                                         ((4, 2, 2, 6), -0.2, 2.5, 1.0)])
def test_free_field_matches_momentum_space(dims, m0, gf, b):
    psi = synth.make_source(dims, 2000)
    U = synth.unit_links(dims)
    got = W.apply_M(U, psi, m0, gf, b)
    ref = mom.apply_M_fft(psi, m0, gf, b)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def _dense(apply, dims):
    lx, ly, lz, lt = dims
    n = lx * ly * lz * lt * 12
    cols = []
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1
        cols.append(apply(e.reshape(lt, lz, ly, lx, 4, 3)).ravel())
    return np.array(cols).T


def test_free_field_singular_values():
    dims, m0, gf, b = (2, 2, 4, 4), -0.05, 3.0, -1.0
    U = synth.unit_links(dims)
    D = _dense(lambda v: W.apply_M(U, v, m0, gf, b), dims)
    sv = np.sort(np.linalg.svd(D, compute_uv=False))
    ref = np.sort(np.repeat(mom.singular_values(dims, m0, gf, b), 12))
    assert np.max(np.abs(sv - ref)) < 1e-13 * ref.max()


@pytest.fixture(scope="module")
def rough():
    dims = (4, 4, 4, 8)
    U = synth.make_links(dims, 0.6, 0.3, 1000)
    return dims, U


def test_links_are_su3(rough):
    _, U = rough
    uu = U @ np.conj(np.swapaxes(U, -1, -2))
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


@pytest.mark.parametrize("cs,ct", [(0.0, 0.0), (1.6 / 3, 1.0)])
def test_gamma5_hermiticity(rough, cs, ct):
    dims, U = rough
    op = Operator(U, -0.05, 3.0, -1.0, cs, ct)
    phi = synth.make_source(dims, 2001)
    psi = synth.make_source(dims, 2002)
    lhs = np.vdot(phi, op.M(psi))
    rhs = np.vdot(dirac.g5(op.M(dirac.g5(phi))), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def _transform_links(U, om):
    out = np.empty_like(U)
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    for mu in range(4):
        out[mu] = om @ U[mu] @ dag(W.link_shift(om, mu, +1))
    return out


@pytest.mark.parametrize("cs,ct", [(0.0, 0.0), (0.5, 0.9)])
def test_gauge_covariance(rough, cs, ct):
    dims, U = rough
    om = synth.make_gauge_transform(dims, 3000)
    Ug = _transform_links(U, om)
    psi = synth.make_source(dims, 2003)
    op = Operator(U, -0.05, 3.0, -1.0, cs, ct)
    opg = Operator(Ug, -0.05, 3.0, -1.0, cs, ct)
    rot = lambda v: np.einsum("...ab,...sb->...sa", om, v)
    lhs = opg.M(rot(psi))
    rhs = rot(op.M(psi))
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3)])
def test_clover_constant_abelian_field(mu, nu):
    """Every plaquette equals exp(i f D): F_{mu nu} = i diag(sin f, -sin f, 0) exactly,
    F_{nu mu} = -F_{mu nu}, and every other plane vanishes."""
    dims = (4, 6, 4, 8)
    n = 1
    U = synth.abelian_plane_links(dims, mu, nu, n)
    f = 2 * np.pi * n / dims[nu]
    want = 1j * np.diag([np.sin(f), -np.sin(f), 0.0])
    F = W.field_strength(U, mu, nu)
    assert np.abs(F - want).max() < 1e-14
    assert np.abs(W.field_strength(U, nu, mu) + want).max() < 1e-14
    for a in range(4):
        for c in range(a + 1, 4):
            if (a, c) != (min(mu, nu), max(mu, nu)):
                assert np.abs(W.field_strength(U, a, c)).max() < 1e-14


def test_clover_plane_weights_isotropic():
    """With c_s = c_t every plane carries the same weight (each spatial plane once)."""
    dims = (6, 6, 6, 6)
    norms = []
    for mu, nu in [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3)]:
        U = synth.abelian_plane_links(dims, mu, nu, 1)
        A = W.clover_field(U, 1.3, 1.3)
        norms.append(np.linalg.norm(A[0, 0, 0, 0]))
    assert np.allclose(norms, norms[0], rtol=1e-14)
    # and the value: |sigma_{mu nu} (x) F| with |F|^2 = 2 sin^2 f, |sigma|^2 = 4
    f = 2 * np.pi / 6
    assert np.isclose(norms[0], 1.3 / 2 * 2 * np.sqrt(2) * np.sin(f), rtol=1e-14)


def test_clover_structure(rough):
    dims, U = rough
    A = W.clover_field(U, 0.7, 1.1)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-14
    g5 = np.kron(dirac.GAMMA5, np.eye(3))
    assert np.abs(A @ g5 - g5 @ A).max() < 1e-14
    # sigma_{mu nu} is traceless in spin: the colour-space partial trace over spin vanishes
    tr_spin = sum(A[..., 3 * s:3 * s + 3, 3 * s:3 * s + 3] for s in range(4))
    assert np.abs(tr_spin).max() < 1e-14
    # time-boundary phase cancels in closed loops
    U2 = U.copy()
    U2[3, -1] *= -1
    assert np.abs(W.clover_field(U2, 0.7, 1.1) - A).max() < 1e-14


def test_clover_gauge_covariance(rough):
    dims, U = rough
    om = synth.make_gauge_transform(dims, 3001)
    Ug = _transform_links(U, om)
    A = W.clover_field(U, 0.7, 1.1)
    Ag = W.clover_field(Ug, 0.7, 1.1)
    O = np.einsum("st,...ab->...satb", np.eye(4), om).reshape(om.shape[:4] + (12, 12))
    assert np.abs(Ag - O @ A @ np.conj(np.swapaxes(O, -1, -2))).max() < 1e-13


def test_clover_small_field_is_linear_in_F():
    """For U = exp(i eps H) with slowly varying H the leading clover term is
    linear in eps, so A(eps)/eps converges as eps -> 0 (checks no spurious O(1)
    terms, e.g. a missing trace subtraction)."""
    dims = (4, 4, 4, 4)
    a1 = W.clover_field(synth.make_links(dims, 1e-4, 1e-4, 7), 1.0, 1.0)
    a2 = W.clover_field(synth.make_links(dims, 2e-4, 2e-4, 7), 1.0, 1.0)
    assert np.linalg.norm(a2 - 2 * a1) < 1e-3 * np.linalg.norm(a2)


def _colour0_low_mode(dims, mu, nu, m0, c):
    """Smallest real part among the near-real eigenvalues of M restricted to colour 0, in
    the constant abelian field of the (mu, nu) plane (one flux quantum per L_nu), with
    gamma_f = 1, periodic time and the SW coefficient c on that plane (c_s for a spatial
    plane, c_t for a plane with t).  Extents of 1 in the other two directions leave them
    at zero momentum, so M is the 2D Wilson operator of the plane plus m0 (and the SW term)."""
    U = synth.abelian_plane_links(dims, mu, nu, 1)
    spatial = mu < 3 and nu < 3
    A = W.clover_field(U, c if spatial else 0.0, 0.0 if spatial else c) if c else None
    lx, ly, lz, lt = dims
    n = lx * ly * lz * lt
    M = np.zeros((4 * n, 4 * n), complex)
    for k in range(4 * n):
        e = np.zeros((n, 4, 3), complex)
        e[k // 4, k % 4, 0] = 1.0
        out = W.apply_M(U, e.reshape(lt, lz, ly, lx, 4, 3), m0, 1.0, 1.0, A).reshape(n, 4, 3)
        assert np.abs(out[..., 1:]).max() < 1e-14  # colour 0 decouples (diagonal links)
        M[:, k] = out[..., 0].ravel()
    ev = np.linalg.eigvals(M)
    near_real = ev[np.abs(ev.imag) < 1e-8]
    return near_real.real.min()


@pytest.mark.parametrize("dims,mu,nu", [((8, 8, 1, 1), 0, 1), ((8, 1, 1, 8), 0, 3),
                                        ((16, 16, 1, 1), 0, 1)])
def test_clover_sign_removes_wilson_mass_shift(dims, mu, nu):
    """The sign of the SW term (Sec. II, the definition of A), pinned by the tree-level
    O(a) improvement it exists for.  In a constant abelian field of flux f per plaquette
    the lowest Landau level of the continuum Dirac operator is a set of exact zero modes.
    The Wilson term lifts them to m0 + f/2 + O(f^2) (its Laplacian equals the squared
    Dirac operator minus the spin-field coupling, which is -|F| on those modes); the SW
    term with coefficient 1 cancels that shift to O(f^2), and with the opposite sign it
    doubles it.  Checked for a spatial plane (c_s) and a plane with t (c_t)."""
    m0 = 0.1
    f = 2 * np.pi / dims[nu]
    wilson = _colour0_low_mode(dims, mu, nu, m0, 0.0) - m0
    improved = _colour0_low_mode(dims, mu, nu, m0, 1.0) - m0
    # Wilson: the O(a) shift f/2 (to within its O(f^2) lattice corrections)
    assert abs(wilson - 0.5 * np.sin(f)) < 0.05 * wilson
    # SW term: the O(a) shift is gone; a flipped sign would give about 2x the Wilson shift
    assert abs(improved) < 0.05 * wilson
