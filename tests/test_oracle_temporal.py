"""Pins of the oracle's temporal preconditioner (Sec. II.A)."""
import numpy as np
import pytest

import synth
from oracle import dirac, wilson as W
from oracle.temporal import Temporal, smw_setup, smw_setup_dag, apply_T
from oracle.dirac import PT_PLUS, PT_MINUS, spin_apply, GAMMA5


@pytest.fixture(scope="module", params=[-1.0, 1.0])
def setup(request):
    b = request.param
    dims = (4, 2, 2, 12)
    U = synth.make_links(dims, 0.5, 0.4, 1000)
    mu = W.mass_term(-0.05, 3.0)
    return dims, U, mu, b, Temporal(U, mu, b)


def test_Tinv_inverts_T(setup):
    dims, U, mu, b, tp = setup
    eta = synth.make_source(dims, 2000)
    assert np.linalg.norm(tp.T(tp.Tinv(eta)) - eta) < 1e-14 * np.linalg.norm(eta)
    assert np.linalg.norm(tp.Tinv(tp.T(eta)) - eta) < 1e-14 * np.linalg.norm(eta)
    assert np.linalg.norm(tp.Tdag(tp.Tdaginv(eta)) - eta) < 1e-14 * np.linalg.norm(eta)


def test_Tdag_is_adjoint_of_T(setup):
    dims, U, mu, b, tp = setup
    a = synth.make_source(dims, 2001)
    c = synth.make_source(dims, 2002)
    assert abs(np.vdot(a, tp.T(c)) - np.vdot(tp.Tdag(a), c)) < 1e-13 * np.linalg.norm(a) * np.linalg.norm(c)


def test_Tinv_matches_dense_line_inverse(setup):
    """Brute force: build the 3Nt x 3Nt matrix of one time line and invert it."""
    dims, U, mu, b, tp = setup
    nt = dims[3]
    eta = synth.make_source(dims, 2003)
    got = tp.Tinv(eta)
    gotd = tp.Tdaginv(eta)
    for (z, y, x) in [(0, 0, 0), (1, 1, 3)]:
        T = np.zeros((3 * nt, 3 * nt), complex)
        for t in range(nt):
            T[3 * t:3 * t + 3, 3 * t:3 * t + 3] = mu * np.eye(3)
            tn = (t + 1) % nt
            ph = b if t == nt - 1 else 1.0
            T[3 * t:3 * t + 3, 3 * tn:3 * tn + 3] -= ph * U[3, t, z, y, x]
        Ti = np.linalg.inv(T)
        Tdi = np.linalg.inv(T.conj().T)
        for s in range(4):
            v = eta[:, z, y, x, s, :].ravel()
            assert np.abs(Ti @ v - got[:, z, y, x, s, :].ravel()).max() < 1e-14
            assert np.abs(Tdi @ v - gotd[:, z, y, x, s, :].ravel()).max() < 1e-14


def test_X_is_partial_polyakov_loop(setup):
    """X(t) = -b mu^-(Nt-t) U(t) U(t+1) ... U(Nt-1), so X(0) = -b mu^-Nt P and
    |X(t)|_F = sqrt(3) mu^-(Nt-t) (eq:cutoff)."""
    dims, U, mu, b, tp = setup
    nt = dims[3]
    X, lam = smw_setup(U[3], mu, b)
    P = U[3, 0]
    for t in range(1, nt):
        P = P @ U[3, t]
    assert np.abs(X[0] - (-b) * mu ** (-nt) * P).max() < 1e-15
    for t in range(nt):
        nrm = np.linalg.norm(X[t], axis=(-2, -1))
        assert np.allclose(nrm, np.sqrt(3) * mu ** (-(nt - t)), rtol=1e-13)
    Xd, _ = smw_setup_dag(U[3], mu, b)
    # the mirrored X' ends on the adjoint of the Polyakov loop based at slice Nt-1,
    # U(Nt-1) U(0) ... U(Nt-2): the same loop started one slice earlier (same trace)
    P1 = U[3, nt - 1]
    for t in range(0, nt - 1):
        P1 = P1 @ U[3, t]
    assert np.abs(Xd[nt - 1] - (-b) * mu ** (-nt) * np.conj(np.swapaxes(P1, -1, -2))).max() < 1e-15
    assert np.allclose(np.trace(P1, axis1=-2, axis2=-1), np.trace(P, axis1=-2, axis2=-1), atol=1e-14)


def test_free_field_T_in_momentum_space():
    dims = (2, 2, 2, 16)
    U = synth.unit_links(dims)
    mu = 1.7
    tp = Temporal(U, mu, -1.0)
    pt = 2 * np.pi * (3 + 0.5) / 16
    t = np.arange(16).reshape(16, 1, 1, 1, 1, 1)
    wave = np.exp(1j * pt * t) * np.ones((16, 2, 2, 2, 4, 3))
    assert np.abs(tp.Tinv(wave) - wave / (mu - np.exp(1j * pt))).max() < 1e-14
    assert np.abs(tp.Tdaginv(wave) - wave / (mu - np.exp(-1j * pt))).max() < 1e-14


def test_mu_minus_Dt_factorises(setup):
    """eqn:dt_clcr: mu - D_t = C_L^-1 C_R^-1, with D_t the oracle's own temporal hop."""
    dims, U, mu, b, tp = setup
    psi = synth.make_source(dims, 2004)
    lhs = mu * psi - W.hop_t(U, psi, b)
    rhs = tp.CL_inv(tp.CR_inv(psi))
    assert np.linalg.norm(lhs - rhs) < 1e-14 * np.linalg.norm(lhs)


def test_CL_CR_inverses_and_gamma5_relation(setup):
    dims, U, mu, b, tp = setup
    psi = synth.make_source(dims, 2005)
    phi = synth.make_source(dims, 2006)
    n = np.linalg.norm(psi)
    assert np.linalg.norm(tp.CL(tp.CL_inv(psi)) - psi) < 1e-14 * n
    assert np.linalg.norm(tp.CR(tp.CR_inv(psi)) - psi) < 1e-14 * n
    # C_L^dagger-1 = gamma5 C_R^-1 gamma5:  <C_L^-1 phi, psi> = <phi, g5 C_R^-1 g5 psi>
    lhs = np.vdot(tp.CL_inv(phi), psi)
    rhs = np.vdot(phi, dirac.g5(tp.CR_inv(dirac.g5(psi))))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # C_R C_L = P- T^-1 + P+ T^dagger^-1
    lhs = tp.CR(tp.CL(psi))
    rhs = spin_apply(PT_MINUS, tp.Tinv(psi)) + spin_apply(PT_PLUS, tp.Tdaginv(psi))
    assert np.linalg.norm(lhs - rhs) < 1e-14 * np.linalg.norm(lhs)


def test_gauge_covariance_of_Tinv(setup):
    dims, U, mu, b, tp = setup
    om = synth.make_gauge_transform(dims, 3002)
    Ug = U.copy()
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    for m in range(4):
        Ug[m] = om @ U[m] @ dag(W.link_shift(om, m, +1))
    tpg = Temporal(Ug, mu, b)
    psi = synth.make_source(dims, 2007)
    rot = lambda v: np.einsum("...ab,...sb->...sa", om, v)
    assert np.linalg.norm(tpg.Tinv(rot(psi)) - rot(tp.Tinv(psi))) < 1e-14 * np.linalg.norm(psi)
    assert np.linalg.norm(tpg.Tdaginv(rot(psi)) - rot(tp.Tdaginv(psi))) < 1e-14 * np.linalg.norm(psi)


@pytest.mark.parametrize("b", [-1.0, 1.0])
@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_cutoff_trick_drops_exactly_the_bounded_terms(b, eps):
    """The cutoff trick (Sec. II.A, eq:cutoff) on a 40-slice line.  Kept slices equal the
    exact inverse (a dense line inverse); on a dropped slice the difference is exactly the
    omitted Woodbury term X(t) q, where q = Lambda chi(0) is the exact psi(0) and X(t) is
    built here from the link products, so it is bounded by sqrt(3) mu^-(Nt-t) |psi(0)| < eps |psi(0)|.
    The mirrored T^dagger^-1 drops X'(t) psi'(Nt-1) at the other end, with sqrt(3) mu^-(t+1)."""
    dims = (2, 2, 2, 40)
    nt = dims[3]
    U = synth.make_links(dims, 0.4, 0.3, 1005)
    mu = W.mass_term(-0.05, 3.0)
    eta = synth.make_source(dims, 2010)
    cut = Temporal(U, mu, b, eps)
    got, gotd = cut.Tinv(eta), cut.Tdaginv(eta)
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    ndrop = 0
    for (z, y, x) in [(0, 0, 0), (1, 0, 1)]:
        T = np.zeros((3 * nt, 3 * nt), complex)
        for t in range(nt):
            T[3 * t:3 * t + 3, 3 * t:3 * t + 3] = mu * np.eye(3)
            ph = b if t == nt - 1 else 1.0
            T[3 * t:3 * t + 3, 3 * ((t + 1) % nt):3 * ((t + 1) % nt) + 3] -= ph * U[3, t, z, y, x]
        Ti, Tdi = np.linalg.inv(T), np.linalg.inv(T.conj().T)
        for s in range(4):
            ex = (Ti @ eta[:, z, y, x, s, :].ravel()).reshape(nt, 3)
            exd = (Tdi @ eta[:, z, y, x, s, :].ravel()).reshape(nt, 3)
            for t in range(nt):
                # X(t) = -b mu^-(Nt-t) U(t) ... U(Nt-1);  X'(t) = -b mu^-(t+1) U(t-1)^dag ... U(0)^dag U(Nt-1)^dag
                Xt = np.eye(3, dtype=complex)
                for j in range(t, nt):
                    Xt = Xt @ U[3, j, z, y, x]
                Xt *= -b * mu ** (-(nt - t))
                Xd = dag(U[3, nt - 1, z, y, x])
                for j in range(0, t):
                    Xd = dag(U[3, j, z, y, x]) @ Xd
                Xd *= -b * mu ** (-(t + 1))
                d = got[t, z, y, x, s] - ex[t]
                dd = gotd[t, z, y, x, s] - exd[t]
                if np.sqrt(3) * mu ** (-(nt - t)) < eps:
                    ndrop += 1
                    assert np.abs(d - Xt @ ex[0]).max() < 1e-14
                    assert np.linalg.norm(d) <= np.sqrt(3) * mu ** (-(nt - t)) * np.linalg.norm(ex[0]) * (1 + 1e-12)
                else:
                    assert np.abs(d).max() < 1e-14
                if np.sqrt(3) * mu ** (-(t + 1)) < eps:
                    assert np.abs(dd - Xd @ exd[nt - 1]).max() < 1e-14
                else:
                    assert np.abs(dd).max() < 1e-14
    # mu = 1.95: sqrt(3) mu^-k < eps from k = 15 (1e-4) and k = 29 (1e-8) on, of 40 slices
    assert ndrop == 2 * 4 * (nt - (15 if eps == 1e-4 else 29) + 1)


def test_cutoff_trick_perturbs_the_ilu_operator_by_order_eps():
    """The App. B sequence built from the cut C_L, C_R stays within a small multiple of eps
    of the exact one, and eps = 0 reproduces it exactly."""
    from oracle.schemes import Operator
    dims = (4, 2, 2, 40)
    U = synth.make_links(dims, 0.35, 0.12, 1000)
    psi = synth.make_source(dims, 2011)
    ex = Operator(U, -0.05, 3.0, -1.0, 1.6 / 3, 1.0)
    ref = ex.tschur_ilu_sequence(psi)
    assert np.array_equal(Operator(U, -0.05, 3.0, -1.0, 1.6 / 3, 1.0, 0.0).tschur_ilu_sequence(psi), ref)
    for eps in (1e-6, 1e-10):
        d = Operator(U, -0.05, 3.0, -1.0, 1.6 / 3, 1.0, eps).tschur_ilu_sequence(psi) - ref
        rel = np.linalg.norm(d) / np.linalg.norm(ref)
        assert 0 < rel < 10 * eps, (eps, rel)
