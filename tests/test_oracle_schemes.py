"""Pins of the oracle's preconditioning schemes (Sec. II.B), solvers and kappa."""
import numpy as np
import pytest

import synth
from oracle import dirac, krylov
from oracle.schemes import Operator, SCHEMES
import _momentum as mom

DIMS = (4, 2, 2, 6)


@pytest.fixture(scope="module", params=["wilson", "clover"])
def op(request):
    U = synth.make_links(DIMS, 0.5, 0.3, 1000)
    if request.param == "wilson":
        return Operator(U, -0.05, 3.0, -1.0)
    return Operator(U, -0.05, 3.0, -1.0, 1.6 / 3.0, 1.0)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_temporal_identity(op):
    """C_L M C_R = I + C_L (A - D_s/gamma_f) C_R (eq:ContaminatedUnprec)."""
    psi = synth.make_source(DIMS, 2000)
    lhs = op.temporal(psi)
    rhs = psi + op.tmp.CL(op.Aop(op.tmp.CR(psi)) - op.Ds(op.tmp.CR(psi)) / op.gamma_f)
    assert _rel(lhs, rhs) < 1e-13


def test_p3_blocks(op):
    """With p3 ordering M^ee = A + mu - D_t and M^eo = -D_s^eo/gamma_f."""
    psi = synth.make_source(DIMS, 2001)
    e, o = op.e3, op.o3
    assert _rel(e * op.M(e * psi), e * (op.Amu(psi) - op.Dt(e * psi))) < 1e-14
    assert _rel(e * op.M(o * psi), -e * op.Ds(o * psi) / op.gamma_f) < 1e-14


def test_p4_blocks(op):
    """With p4 ordering M^ee = A + mu (hops always change the 4D parity)."""
    psi = synth.make_source(DIMS, 2002)
    e = op.e4
    assert _rel(e * op.M(e * psi), e * op.Amu(psi)) < 1e-14


def test_tschur_product_equals_closed_form_and_ilu_sequence(op):
    psi = synth.make_source(DIMS, 2003)
    lit = op.tschur(psi)
    assert _rel(op.tschur_closed_form(psi), lit) < 1e-13
    assert _rel(op.tschur_ilu_sequence(psi), lit) < 1e-13
    if not op.clover:
        # eq:TPrecFull: diag(1, 1 - D-bar^oe D-bar^eo / gamma_f^2)
        e, o = op.e3, op.o3
        want = e * psi + o * psi - op.Dbar_oe(op.Dbar_eo(o * psi)) / op.gamma_f ** 2
        assert _rel(want, lit) < 1e-13


def test_mee_inverse(op):
    """The dense even-block inverse: M^ee (M^ee)^-1 = 1 on even p3 sites, and for Wilson
    fermions (M^ee)^-1 = C_R C_L, the scan form of Sec. II.A (mu - D_t = C_L^-1 C_R^-1)."""
    psi = synth.make_source(DIMS, 2010)
    e = op.e3
    f = op.Mee_inv(psi)
    assert _rel(e * op.M(f), e * psi) < 1e-13
    if not op.clover:
        assert _rel(f, e * op.tmp.CR(op.tmp.CL(e * psi))) < 1e-13


def test_tschur3d_wilson_is_tprecfull(op):
    """With A = 0 the exact 3D-Schur scheme is eq:TPrecFull (the ILU scheme's Wilson form)."""
    psi = synth.make_source(DIMS, 2011)
    if op.clover:
        # the clover term makes the two schemes differ
        assert _rel(op.tschur3d(psi), op.tschur(psi)) > 1e-3
    else:
        assert _rel(op.tschur3d(psi), op.tschur(psi)) < 1e-13


def test_schur3d_complement_inverts_odd_block(op):
    """Brute force: S_o applied to the odd part of M^-1 psi_o returns psi_o (dense LU)."""
    psi = op.o3 * synth.make_source(DIMS, 2012)
    x = np.linalg.solve(_dense_M(op), psi.ravel()).reshape(psi.shape)
    assert _rel(op.schur3d_S(op.o3 * x), psi) < 1e-12


def test_fullsw_T_inverse(op):
    """The whole-lattice T^-1 of TEMPORAL_FULLSW: (A + mu - D_t) T^-1 psi = psi on every site,
    and for Wilson fermions T^-1 = C_R C_L, the scan form of Sec. II.A, while with a clover
    term it differs from it; Mt = 1 - T^-1 D_s / gamma_f then follows from the definitions."""
    psi = synth.make_source(DIMS, 2013)
    f = op.T_inv(psi)
    assert _rel(op.Amu(f) - op.Dt(f), psi) < 1e-13
    scan = op.tmp.CR(op.tmp.CL(psi))
    if op.clover:
        assert _rel(f, scan) > 1e-3
    else:
        assert _rel(f, scan) < 1e-13
    # M = T - D_s / gamma_f, so T^-1 M = Mt
    assert _rel(op.T_inv(op.M(psi)), op.fullsw(psi)) < 1e-13


def test_schur4d_ldu(op):
    """L diag(M^ee, S-hat) U = M, with L^-1 = S_L and U^-1 = S_R as applied."""
    psi = synth.make_source(DIMS, 2004)
    # S_L M S_R psi == Mt psi
    assert _rel(op.schur4d_SL(op.M(op.schur4d_SR(psi))), op.schur4d(psi)) < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_prec_is_SL_M_SR(op, scheme):
    psi = synth.make_source(DIMS, 2005)
    assert _rel(op.prepare_source(scheme, op.M(op.reconstruct(scheme, psi))),
                op.prec(scheme, psi)) < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_gamma5_hermiticity_of_prec(op, scheme):
    phi = synth.make_source(DIMS, 2006)
    psi = synth.make_source(DIMS, 2007)
    lhs = np.vdot(phi, op.prec(scheme, psi))
    rhs = np.vdot(op.prec_dag(scheme, phi), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def _dense_M(op):
    lx, ly, lz, lt = op.dims
    n = lx * ly * lz * lt * 12
    cols = []
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1
        cols.append(op.M(e.reshape(lt, lz, ly, lx, 4, 3)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("solver", ["bicgstab", "cgnr"])
def test_solve_matches_dense_lu(op, scheme, solver):
    """Brute force: the preconditioned solve reproduces x = M^-1 eta from dense LU."""
    eta = synth.make_source(DIMS, 2008)
    x_ref = np.linalg.solve(_dense_M(op), eta.ravel()).reshape(eta.shape)
    x, info = krylov.solve(op, scheme, eta, solver, 1e-11)
    assert info["true_rel_resid"] <= 1e-11
    assert _rel(x, x_ref) < 1e-9


def test_krylov_on_dense_matrix():
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xr = np.linalg.solve(A, b)
    x1, _ = krylov.bicgstab(lambda v: A @ v, b, 1e-12)
    x2, info = krylov.cgnr(lambda v: A @ v, lambda v: A.conj().T @ v, b, 1e-12)
    assert _rel(x1, xr) < 1e-10 and _rel(x2, xr) < 1e-10
    sv = np.linalg.svd(A, compute_uv=False)
    lmin, lmax, kap = krylov.lanczos_kappa(info["alphas"], info["betas"])
    assert np.isclose(kap, (sv.max() / sv.min()) ** 2, rtol=1e-6)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_free_field_kappa(scheme):
    """Lanczos kappa of each scheme on 4^3 x 16, xi = 3, against momentum space."""
    dims = (4, 4, 4, 16)
    op = Operator(synth.unit_links(dims), -0.05, 3.0, -1.0)
    eta = synth.make_source(dims, 2009)
    et = op.prepare_source(scheme, eta)
    mask, _ = op.solve_subspace(scheme)
    if mask is None:
        A = lambda v: op.prec(scheme, v)
        Ad = lambda v: op.prec_dag(scheme, v)
    else:
        A = lambda v: mask * op.prec(scheme, mask * v)
        Ad = lambda v: mask * op.prec_dag(scheme, mask * v)
        et = mask * et
    _, info = krylov.cgnr(A, Ad, et, 1e-12)
    _, _, kap = krylov.lanczos_kappa(info["alphas"], info["betas"])
    ref = mom.kappa_free(dims, -0.05, 3.0, -1.0, scheme)
    assert abs(kap / ref - 1) < 0.01, (kap, ref)
