"""GPU parity: every C-ABI apply against the FP64 oracle, element by element.

Tolerances (relative l2 over the whole field):
  F64  1e-12   (the operators are exact re-expressions; rounding only)
  F32  3e-6 single kernels, 2e-5 composites   (FP32 rounding, ~2^-24 per op times depth)
  F16N 4e-3 single kernels, 1.5e-2 composites (FP16 storage, 2^-11 relative per stored half
       spinor, scaled by its largest component)
Beside the global l2, every comparison bounds the worst site: max over sites of |error(x)|
divided by max over sites of |reference(x)| must stay below twice the same tolerance, so an
error confined to a few sites (which the global l2 dilutes by the square root of the volume)
fails as well.
Lattices span several workgroups, ragged line counts, time extents that are not
powers of two, and the scan's fast path (time extents that are multiples of 16,
up to 16 wavefront segments of 16 chunks per line).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dirac, wilson as W
from oracle.schemes import Operator as OOp, SCHEMES
from oracle import krylov, force as oforce

pytestmark = pytest.mark.gpu

TOL = {"F64": (1e-12, 1e-12), "F32": (3e-6, 2e-5), "F16N": (4e-3, 1.5e-2)}

CASES = {
    # name: dims, eps_s, eps_t, xi, m0, csw_s, csw_t, bc
    "wilson_4x16": ((4, 4, 4, 16), 0.3, 0.1, 3.0, -0.05, 0.0, 0.0, -1),
    "clover_8x32": ((8, 8, 8, 32), 0.35, 0.12, 3.5, -0.05, 1.6, 1.0, -1),
    "clover_ragged": ((6, 4, 2, 10), 0.5, 0.3, 2.0, 0.1, 1.2, 0.9, -1),
    "clover_periodic": ((4, 6, 4, 12), 0.4, 0.2, 5.0, -0.05, 1.6, 1.0, 1),
    # long lines: 16 wavefront segments of 16 chunks (the 256-slice benchmark shape)
    "clover_long": ((4, 2, 2, 256), 0.4, 0.1, 6.0, -0.01, 1.6, 1.0, -1),
    # 3 segments, many tiles per workgroup
    "clover_lt48": ((6, 6, 4, 48), 0.35, 0.12, 3.5, -0.01, 1.6, 1.0, -1),
    # short lines: a workgroup of 16 lines x 6 slices has fewer threads than the 16 x 9 closure
    # entries it stages
    "clover_lt6": ((4, 4, 2, 6), 0.4, 0.2, 2.5, -0.05, 1.6, 1.0, -1),
    # U(3) spatial links (a random U(1) phase on each): not SU(3), so the reduced-precision
    # kernels read all nine link entries instead of rebuilding the third row
    "clover_u3_spatial": ((4, 4, 4, 16), 0.35, 0.12, 3.0, -0.05, 1.6, 1.0, -1, "u1_spatial"),
}


def _links(dims, es, et, variant):
    U = synth.make_links(dims, es, et, 1000)
    if variant == "u1_spatial":
        rng = np.random.default_rng(77)
        ph = np.exp(2j * np.pi * rng.random((3,) + tuple(reversed(dims)) + (1, 1)))
        U[:3] *= ph
    return U


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _site_rel(a, b):
    """max_x |a(x) - b(x)| / max_x |b(x)| over sites (the last two axes are one site's
    spin-colour components, or one link's colour matrix)."""
    a = np.asarray(a)
    b = np.asarray(b)
    n = a.shape[-1] * a.shape[-2]
    da = np.linalg.norm((a - b).reshape(-1, n), axis=1)
    nb = np.linalg.norm(b.reshape(-1, n), axis=1)
    return float(da.max() / nb.max())


def _close(a, b, tol, what=""):
    err = _rel(a, b)
    assert err < tol, f"{what}: relative error {err:.3e} >= {tol:.1e}"
    serr = _site_rel(a, b)
    assert serr < 2 * tol, f"{what}: worst-site relative error {serr:.3e} >= {2 * tol:.1e}"


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_0910_0992_amd import Operator
    dims, es, et, xi, m0, cs, ct, bc, *variant = CASES[request.param]
    U = _links(dims, es, et, variant[0] if variant else None)
    c_s = cs / xi
    oop = OOp(U, m0, xi, float(bc), c_s, ct)
    gop = Operator(torch.from_numpy(U).cuda(), m0, xi, c_s, ct, bc)
    eta = synth.make_source(dims, 2000)
    print(f"[case] {request.param} dims={dims}", flush=True)
    yield dict(name=request.param, dims=dims, U=U, oop=oop, gop=gop, eta=eta,
               teta=torch.from_numpy(eta).cuda(), xi=xi, m0=m0, bc=bc, cache={})
    gop.close()


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
def test_apply_M(case, prec):
    o, g = case["oop"], case["gop"]
    tol = TOL[prec][0] * (1 if prec == "F64" else 2)
    _close(_np(g.apply_M(case["teta"], prec)), o.M(case["eta"]), tol, '_np(g.apply_M(case["teta"], prec)), o.M(')
    _close(_np(g.apply_M(case["teta"], prec, dagger=True)), o.Mdag(case["eta"]), tol, '_np(g.apply_M(case["teta"], prec, dagger')


@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
def test_apply_Ds(case, prec):
    o, g = case["oop"], case["gop"]
    _close(_np(g.apply_Ds(case["teta"], prec)), o.Ds(case["eta"]), TOL[prec][0] * (1 if prec == "F64" else 2), '_np(g.apply_Ds(case["teta"], prec)), o.D')


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_apply_clover(case, prec):
    o, g = case["oop"], case["gop"]
    tol = TOL[prec][0] * (1 if prec == "F64" else 2)
    if o.clover:
        _close(_np(g.apply_clover(case["teta"], prec, 0)), o.Aop(case["eta"]), tol, '_np(g.apply_clover(case["teta"], prec, 0')
    _close(_np(g.apply_clover(case["teta"], prec, 1)), o.Amu(case["eta"]), tol, '_np(g.apply_clover(case["teta"], prec, 1')
    _close(_np(g.apply_clover(case["teta"], prec, -1)), o.Amu_inv(case["eta"]), tol, '_np(g.apply_clover(case["teta"], prec, -')


@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
def test_temporal_inverses(case, prec):
    o, g = case["oop"], case["gop"]
    e, te = case["eta"], case["teta"]
    tol = TOL[prec][0]
    _close(_np(g.apply_Tinv(te, prec)), o.tmp.Tinv(e), tol, '_np(g.apply_Tinv(te, prec)), o.tmp.Tinv(')
    _close(_np(g.apply_Tinv(te, prec, dagger=True)), o.tmp.Tdaginv(e), tol, '_np(g.apply_Tinv(te, prec, dagger=True))')
    _close(_np(g.apply_CL(te, prec)), o.tmp.CL(e), tol, '_np(g.apply_CL(te, prec)), o.tmp.CL(e)')
    _close(_np(g.apply_CR(te, prec)), o.tmp.CR(e), tol, '_np(g.apply_CR(te, prec)), o.tmp.CR(e)')


@pytest.mark.parametrize("prec", ["F32", "F16N"])
def test_point_source_reduced_precision(case, prec):
    """A point source: along a long line T^-1 decays as mu^-t far below the FP32 normal
    range (mu^-256 ~ 5e-42 on the 256-slice lattice); the FP16 form must stay finite and
    accurate there."""
    o, g = case["oop"], case["gop"]
    e = synth.make_point_source(case["dims"], 1, 2, (1, 0, 1, 2))
    te = torch.from_numpy(e).cuda()
    for got, want, what in [(g.apply_Tinv(te, prec), o.tmp.Tinv(e), "T^-1"),
                            (g.apply_Tinv(te, prec, dagger=True), o.tmp.Tdaginv(e), "T^dag^-1"),
                            (g.prepare_source(te, "TEMPORAL_SCHUR", prec), o.prepare_source("TEMPORAL_SCHUR", e),
                             "prepare")]:
        got = _np(got)
        assert np.all(np.isfinite(got)), what
        _close(got, want, TOL[prec][1], what)


@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_apply_prec(case, scheme, prec):
    if scheme == "SCHUR4D" and prec == "F16N":
        pytest.skip("the 4D Schur baseline runs in F64/F32")
    if scheme in ("TEMPORAL_SCHUR3D", "TEMPORAL_FULLSW") and prec == "F16N":
        pytest.skip("the exact block-LU inverse runs in F64 and F32")
    o, g = case["oop"], case["gop"]
    e, te = case["eta"], case["teta"]
    tol = TOL[prec][1]
    _close(_np(g.apply_prec(te, scheme, prec)), o.prec(scheme, e), tol, '_np(g.apply_prec(te, scheme, prec)), o.p')
    _close(_np(g.apply_prec(te, scheme, prec, dagger=True)), o.prec_dag(scheme, e), tol, '_np(g.apply_prec(te, scheme, prec, dagge')
    _close(_np(g.prepare_source(te, scheme, prec)), o.prepare_source(scheme, e), tol, '_np(g.prepare_source(te, scheme, prec)),')
    _close(_np(g.reconstruct(te, scheme, prec)), o.reconstruct(scheme, e), tol, '_np(g.reconstruct(te, scheme, prec)), o.')


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("solver", ["BICGSTAB", "CGNR"])
def test_solve_f64(case, scheme, solver):
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme=scheme, solver=solver, prec="F64", tol=1e-10)
    xn = _np(x)
    true = np.linalg.norm(case["eta"] - o.M(xn)) / np.linalg.norm(case["eta"])
    assert info["true_rel_resid"] <= 1e-10 and true <= 1.05e-10, (info, true)
    # oracle solve of the same system; the two solutions agree within kappa * residual
    if "xo" not in case["cache"]:
        case["cache"]["xo"], _ = krylov.solve(o, "TEMPORAL_SCHUR", case["eta"], "bicgstab", 1e-12)
    _close(xn, case["cache"]["xo"], 1e-6, 'xn, case["cache"]["xo"]')


@pytest.mark.parametrize("prec", ["F32", "F16N"])
@pytest.mark.parametrize("scheme", ["TEMPORAL_SCHUR", "UNPREC", "TEMPORAL"])
def test_solve_mixed(case, prec, scheme):
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme=scheme, prec=prec, tol=1e-10)
    xn = _np(x)
    true = np.linalg.norm(case["eta"] - o.M(xn)) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    assert info["outer_iters"] >= 2  # the inner precision alone cannot reach 1e-10


@pytest.mark.parametrize("prec", ["F32", "F16N"])
def test_solve_from_initial_guess(case, prec):
    """A mixed solve started from x0 (use_x0) reaches the target from there: from a slightly
    perturbed solution in fewer iterations than from zero, from the solution itself at once."""
    o, g = case["oop"], case["gop"]
    x_ref, i_ref = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec=prec, tol=1e-10)
    rng = np.random.default_rng(5)
    noise = rng.standard_normal(x_ref.shape) + 1j * rng.standard_normal(x_ref.shape)
    xr = _np(x_ref)
    x0 = xr + 1e-6 * np.linalg.norm(xr) / np.linalg.norm(noise) * noise
    x, info = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec=prec, tol=1e-10,
                      x0=torch.from_numpy(x0).cuda())
    true = np.linalg.norm(case["eta"] - o.M(_np(x))) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    assert info["iters"] < i_ref["iters"], (info, i_ref)
    x2, info2 = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec=prec, tol=1e-10, x0=x_ref)
    assert info2["iters"] <= 2, info2
    true2 = np.linalg.norm(case["eta"] - o.M(_np(x2))) / np.linalg.norm(case["eta"])
    assert true2 <= 1.05e-10


@pytest.mark.parametrize("delta", [0.005, 0.05])
def test_solve_reliable_update_threshold(case, delta):
    """Any reliable-update threshold reaches the FP64 target.  An update follows a drop of the
    recursive residual to delta times its running maximum, so a larger delta folds the
    correction into FP64 at least as often."""
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec="F16N", tol=1e-10, inner_tol=delta)
    true = np.linalg.norm(case["eta"] - o.M(_np(x))) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    if delta == 0.05:
        _, tight = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec="F16N", tol=1e-10,
                           inner_tol=0.005)
        assert info["outer_iters"] >= tight["outer_iters"], (info, tight)


@pytest.mark.parametrize("prec", ["F32", "F16N"])
def test_solve_iteration_limit(case, prec):
    """A mixed solve cut off after a few iterations reports non-convergence and returns the
    best FP64 iterate it has: finite, and no worse than x = 0."""
    from paper_0910_0992_amd import _lib as L
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", prec=prec, tol=1e-10, max_iter=4,
                      raise_on_noconv=False)
    assert info["status"] == L.TP_ENOCONV, info
    xn = _np(x)
    assert np.all(np.isfinite(xn))
    true = np.linalg.norm(case["eta"] - o.M(xn)) / np.linalg.norm(case["eta"])
    assert true <= 1.0 + 1e-12, (info, true)
    assert info["iters"] <= 4 + 1, info


@pytest.mark.parametrize("prec", ["F32", "F16N"])
@pytest.mark.parametrize("scheme", ["TEMPORAL_SCHUR", "TEMPORAL", "UNPREC", "SCHUR4D"])
def test_solve_multi(case, prec, scheme):
    """Batched right-hand sides (lockstep BiCGStab, or one after another where the scheme
    has no batched path): each solution meets the oracle's true residual, a zero source
    gives zero, and the batch agrees with the single-source solve."""
    if scheme == "SCHUR4D" and prec == "F16N":
        pytest.skip("SCHUR4D takes F64 and F32")
    o, g = case["oop"], case["gop"]
    etas = [case["eta"], synth.make_source(case["dims"], 2004), np.zeros_like(case["eta"]),
            synth.make_point_source(case["dims"], 1, 2, (1, 0, 1, 2))]
    xs, infos = g.solve_multi([torch.from_numpy(e).cuda() for e in etas], scheme=scheme, prec=prec,
                              tol=1e-10)
    xs = _np(xs)
    for k, e in enumerate(etas):
        if not np.any(e):
            assert not np.any(xs[k]) and infos[k]["true_rel_resid"] == 0.0
            continue
        true = np.linalg.norm(e - o.M(xs[k])) / np.linalg.norm(e)
        assert true <= 1.05e-10, (k, infos[k], true)
        assert infos[k]["true_rel_resid"] <= 1e-10, (k, infos[k])
    x1, _ = g.solve(torch.from_numpy(etas[1]).cuda(), scheme=scheme, prec=prec, tol=1e-10)
    _close(xs[1], _np(x1), 1e-7, "batched vs single solve")


@pytest.mark.parametrize("prec", ["F32", "F16N"])
def test_solve_mixed_cgnr(case, prec):
    """CGNR with FP64 defect correction in the reduced precision reaches the FP64 target."""
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="TEMPORAL_SCHUR", solver="CGNR", prec=prec, tol=1e-10)
    true = np.linalg.norm(case["eta"] - o.M(_np(x))) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    assert info["outer_iters"] >= 2


def test_solve_multi_from_initial_guess(case):
    """A batch started from its own solutions needs almost no work and stays converged."""
    o, g = case["oop"], case["gop"]
    etas = [torch.from_numpy(case["eta"]).cuda(),
            torch.from_numpy(synth.make_source(case["dims"], 2004)).cuda()]
    xs, _ = g.solve_multi(etas, scheme="TEMPORAL_SCHUR", prec="F16N", tol=1e-10)
    xs2, infos = g.solve_multi(etas, scheme="TEMPORAL_SCHUR", prec="F16N", tol=1e-10, x0=xs)
    for k in range(2):
        assert infos[k]["iters"] <= 2, infos[k]
        e = _np(etas[k])
        true = np.linalg.norm(e - o.M(_np(xs2[k]))) / np.linalg.norm(e)
        assert true <= 1.05e-10, (k, infos[k], true)


def test_solve_schur4d_f32_mixed(case):
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="SCHUR4D", prec="F32", tol=1e-10)
    true = np.linalg.norm(case["eta"] - o.M(_np(x))) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)


def test_force_matches_oracle(case):
    """Link gradient: the hopping part alone (TP_FORCE_HOPPING_ONLY) and the whole gradient
    with the SW term's link dependence, raw and su(3)-projected."""
    o, g = case["oop"], case["gop"]
    x = synth.make_source(case["dims"], 2001)
    lam = synth.make_source(case["dims"], 2002)
    tx, tl = torch.from_numpy(x).cuda(), torch.from_numpy(lam).cuda()
    raw_h, G_h = oforce.link_gradient(o, x, lam)
    _close(_np(g.force(tx, tl, projected=False, hopping_only=True)), raw_h, 1e-12, "hopping raw")
    _close(_np(g.force(tx, tl, projected=True, hopping_only=True)), G_h, 1e-12, "hopping projected")
    raw_o, G_o = oforce.full_link_gradient(o, x, lam)
    _close(_np(g.force(tx, tl, projected=False)), raw_o, 1e-12, "full raw")
    _close(_np(g.force(tx, tl, projected=True)), G_o, 1e-12, "full projected")


def test_plaquette(case):
    U = case["U"]
    g = case["gop"]
    ps, pt = g.plaquette()
    want = []
    for planes in ([(0, 1), (0, 2), (1, 2)], [(0, 3), (1, 3), (2, 3)]):
        acc = 0.0
        for mu, nu in planes:
            l = (U[mu] @ W.link_shift(U[nu], mu, 1) @ np.conj(np.swapaxes(W.link_shift(U[mu], nu, 1), -1, -2))
                 @ np.conj(np.swapaxes(U[nu], -1, -2)))
            acc += np.trace(l, axis1=-2, axis2=-1).real.mean() / 3
        want.append(acc / 3)
    assert abs(ps - want[0]) < 1e-12 and abs(pt - want[1]) < 1e-12


def test_gauge_rejects_nonunitary_time_links():
    """The p3 operators rotate by the time-line products W^dag, a gauge rotation only when
    the time links are unitary; a non-unitary time link is refused at set-up."""
    from paper_0910_0992_amd import Operator
    from paper_0910_0992_amd._lib import TprecError
    dims = (4, 4, 4, 8)
    U = synth.make_links(dims, 0.3, 0.1, 5)
    U[3, 2, 1, 0, 3] *= 1.01
    with pytest.raises(TprecError, match="unitary"):
        Operator(torch.from_numpy(U).cuda(), -0.05, 3.0, 0.5, 1.0, -1)
    # an overall U(1) phase on the time links is still unitary and accepted
    U = synth.make_links(dims, 0.3, 0.1, 5)
    U[3] *= np.exp(0.3j)
    Operator(torch.from_numpy(U).cuda(), -0.05, 3.0, 0.5, 1.0, -1).close()


@pytest.mark.parametrize("dev", [3e-11, 3e-7])
def test_nearly_su3_spatial_links(dev):
    """Spatial links off SU(3) by `dev` (a non-unitary factor 1 + dev*i*H per link): the FP64
    hops read two rows only when every link is SU(3) to 1e-13 and the reduced-precision hops
    when it is to 1e-9, so FP64 stays within 1e-12 and F32/F16N within their bounds either way
    (a rebuilt third row would carry an error of order dev)."""
    from paper_0910_0992_amd import Operator
    dims = (4, 4, 4, 8)
    U = synth.make_links(dims, 0.35, 0.12, 11)
    rng = np.random.default_rng(12)
    h = rng.standard_normal((3,) + U.shape[1:]) + 1j * rng.standard_normal((3,) + U.shape[1:])
    h = 0.5 * (h + np.conj(np.swapaxes(h, -1, -2)))
    U[:3] = U[:3] @ (np.eye(3) + 1j * dev * h)
    o = OOp(U, -0.05, 3.0, -1.0, 0.5, 1.0)
    g = Operator(torch.from_numpy(U).cuda(), -0.05, 3.0, 0.5, 1.0, -1)
    try:
        e = synth.make_source(dims, 2000)
        te = torch.from_numpy(e).cuda()
        for prec in ("F64", "F32", "F16N"):
            tol = TOL[prec][0] * (1 if prec == "F64" else 2)
            _close(_np(g.apply_M(te, prec)), o.M(e), tol, f"M {prec}")
            _close(_np(g.apply_Ds(te, prec)), o.Ds(e), tol, f"D_s {prec}")
        _close(_np(g.apply_prec(te, "TEMPORAL_SCHUR", "F64")), o.prec("TEMPORAL_SCHUR", e), TOL["F64"][1],
               "temporal + 3D-ILU F64")
    finally:
        g.close()


# Shapes on which the site kernels visit tiles in their XCD-aware order (time extent a
# multiple of 64 up to 512, Lx/2 a multiple of 4): 1, 2, 4 and 8 blocks per tile, two tiles
# per x row and several z blocks.
ORDER_SHAPES = [(16, 2, 12, 64), (16, 2, 12, 128), (8, 4, 4, 256), (8, 2, 2, 512)]


@pytest.mark.parametrize("dims", ORDER_SHAPES)
def test_site_kernels_in_tile_order(dims):
    from paper_0910_0992_amd import Operator
    xi, m0, cs, ct = 3.5, -0.05, 1.6, 1.0
    U = synth.make_links(dims, 0.35, 0.12, 1000)
    oop = OOp(U, m0, xi, -1.0, cs / xi, ct)
    gop = Operator(torch.from_numpy(U).cuda(), m0, xi, cs / xi, ct, -1)
    eta = synth.make_source(dims, 2000)
    teta = torch.from_numpy(eta).cuda()
    print(f"[order] dims={dims}", flush=True)
    try:
        m = oop.M(eta)
        ts = oop.tschur(eta)
        for prec in ("F64", "F32", "F16N"):
            t1 = TOL[prec][0] * (1 if prec == "F64" else 2)
            _close(_np(gop.apply_M(teta, prec)), m, t1, f"M {prec}")
            _close(_np(gop.apply_Ds(teta, prec)), oop.Ds(eta), t1, f"D_s {prec}")
            _close(_np(gop.apply_prec(teta, "TEMPORAL_SCHUR", prec=prec)), ts, TOL[prec][1],
                   f"TEMPORAL_SCHUR {prec}")
    finally:
        gop.close()


@pytest.mark.parametrize("scheme", ["TEMPORAL_SCHUR3D", "TEMPORAL_FULLSW"])
def test_block_lu_schemes_reject_f16n(case, scheme):
    from paper_0910_0992_amd._lib import TprecError
    g = case["gop"]
    with pytest.raises(TprecError, match="F64 and F32"):
        g.apply_prec(case["teta"], scheme, "F16N")
    with pytest.raises(TprecError, match="F64 and F32"):
        g.solve(case["teta"], scheme=scheme, prec="F16N", tol=1e-10)


def test_schur3d_solve_mixed_f32(case):
    """FP32 inner solves with the FP32-rounded factors, FP64 reliable updates, to 1e-10."""
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="TEMPORAL_SCHUR3D", prec="F32", tol=1e-10)
    xn = _np(x)
    true = np.linalg.norm(case["eta"] - o.M(xn)) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    assert info["outer_iters"] >= 2


def test_schur3d_even_block_inverse(case):
    """The even half of the prepared source is (M^ee)^-1 eta_e: M^ee applied to it (the even
    block of M, from the separately checked M apply) returns eta_e."""
    o, g = case["oop"], case["gop"]
    e = o.e3
    f = _np(g.prepare_source(case["teta"], "TEMPORAL_SCHUR3D", "F64"))
    back = _np(g.apply_M(torch.from_numpy(e * f).cuda(), "F64"))
    _close(e * back, e * case["eta"], 1e-12, "M^ee (M^ee)^-1 eta_e")


def test_fullsw_solve_mixed_f32(case):
    """Full SW temporal preconditioning on the whole lattice: FP32 inner solves with the
    FP32-rounded factors of both parities and FP64 reliable updates, single and batched
    (two right-hand sides in lockstep), to 1e-10."""
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme="TEMPORAL_FULLSW", prec="F32", tol=1e-10)
    true = np.linalg.norm(case["eta"] - o.M(_np(x))) / np.linalg.norm(case["eta"])
    assert true <= 1.05e-10, (info, true)
    assert info["outer_iters"] >= 2
    e2 = synth.make_source(case["dims"], 2004)
    xs, infos = g.solve_multi([case["teta"], torch.from_numpy(e2).cuda()], scheme="TEMPORAL_FULLSW",
                              prec="F32", tol=1e-10)
    xs = _np(xs)
    for k, e in enumerate([case["eta"], e2]):
        true = np.linalg.norm(e - o.M(xs[k])) / np.linalg.norm(e)
        assert true <= 1.05e-10, (k, infos[k], true)


def test_fullsw_T_inverse(case):
    """The prepared source of TEMPORAL_FULLSW is T^-1 eta with T = A + mu - D_t on both
    parities: T = M + D_s / gamma_f applied to it (the separately checked M and D_s applies)
    returns eta, in FP64 and with the FP32 factors."""
    g, xi = case["gop"], case["xi"]
    for prec, tol in (("F64", TOL["F64"][1]), ("F32", TOL["F32"][1])):
        f = g.prepare_source(case["teta"], "TEMPORAL_FULLSW", prec)
        back = _np(g.apply_M(f, "F64")) + _np(g.apply_Ds(f, "F64")) / xi
        _close(back, case["eta"], tol, f"T T^-1 eta ({prec})")


@pytest.mark.parametrize("scheme,prec", [("TEMPORAL_SCHUR", "F16N"), ("TEMPORAL_SCHUR", "F64"),
                                         ("SCHUR4D", "F64"), ("TEMPORAL_SCHUR3D", "F32"),
                                         ("TEMPORAL_FULLSW", "F32")])
def test_solve_dagger(case, scheme, prec):
    """M^dagger x = eta (tp_solve with dagger): the oracle's M^dagger residual of the solution,
    single and batched."""
    o, g = case["oop"], case["gop"]
    x, info = g.solve(case["teta"], scheme=scheme, prec=prec, tol=1e-10, dagger=True)
    true = np.linalg.norm(case["eta"] - o.Mdag(_np(x))) / np.linalg.norm(case["eta"])
    assert info["true_rel_resid"] <= 1e-10 and true <= 1.05e-10, (info, true)
    e2 = synth.make_source(case["dims"], 2004)
    xs, infos = g.solve_multi([case["teta"], torch.from_numpy(e2).cuda()], scheme=scheme, prec=prec,
                              tol=1e-10, dagger=True)
    xs = _np(xs)
    for k, e in enumerate([case["eta"], e2]):
        true = np.linalg.norm(e - o.Mdag(xs[k])) / np.linalg.norm(e)
        assert true <= 1.05e-10, (k, infos[k], true)


def test_allocator_accounting(case):
    """With torch's caching allocator registered (the binding's default) every device byte
    the library holds is torch memory, and closing the operator returns all of it; an
    operator on hipMalloc gives bit-identical results."""
    from paper_0910_0992_amd import Operator
    dims, xi, bc = case["dims"], case["xi"], case["bc"]
    o = case["oop"]
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    gt = Operator(torch.from_numpy(case["U"]).cuda(), case["m0"], xi, o.c_s, o.c_t, bc)
    gh = Operator(torch.from_numpy(case["U"]).cuda(), case["m0"], xi, o.c_s, o.c_t, bc, allocator="hip")
    try:
        yt = gt.apply_prec(case["teta"], "TEMPORAL_SCHUR", "F16N")
        yh = gh.apply_prec(case["teta"], "TEMPORAL_SCHUR", "F16N")
        assert torch.equal(yt, yh)
        torch.cuda.synchronize()
        lib = gt.device_bytes()
        held = torch.cuda.memory_allocated() - m0 - 2 * yt.numel() * yt.element_size()
        # torch rounds each block up (a large block keeps a remainder of up to 1 MB unsplit)
        assert lib > 0 and lib <= held <= 1.05 * lib + 8 * 2 ** 20, (lib, held)
    finally:
        gt.close()
        gh.close()
    del yt, yh
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0


@pytest.mark.parametrize("scheme", SCHEMES)
def test_kappa_free_field(scheme):
    """The library's Lanczos estimate of kappa(Mt^dag Mt) from its CGNR coefficients, on the
    free field 4^3x16 (xi = 3, m0 = -0.05), against the momentum-space closed form."""
    import _momentum as mom
    from paper_0910_0992_amd import Operator
    dims = (4, 4, 4, 16)
    g = Operator(torch.from_numpy(synth.unit_links(dims)).cuda(), -0.05, 3.0, 0.0, 0.0, -1)
    try:
        eta = torch.from_numpy(synth.make_source(dims, 2009)).cuda()
        _, info = g.solve(eta, scheme=scheme, solver="CGNR", prec="F64", tol=1e-12, estimate_kappa=True)
    finally:
        g.close()
    ref = mom.kappa_free(dims, -0.05, 3.0, -1.0, scheme)
    assert abs(info["kappa_est"] / ref - 1) < 0.01, (scheme, info["kappa_est"], ref)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_kappa_interacting(scheme):
    """kappa on random clover links (4^3x16): the library's estimate against the oracle's
    Lanczos estimate from its own CGNR on the same prepared source."""
    from paper_0910_0992_amd import Operator
    dims, xi, m0 = (4, 4, 4, 16), 3.0, -0.05
    U = synth.make_links(dims, 0.35, 0.12, 1000)
    oop = OOp(U, m0, xi, -1.0, 1.6 / xi, 1.0)
    eta = synth.make_source(dims, 2000)
    g = Operator(torch.from_numpy(U).cuda(), m0, xi, 1.6 / xi, 1.0, -1)
    try:
        _, info = g.solve(torch.from_numpy(eta).cuda(), scheme=scheme, solver="CGNR", prec="F64",
                          tol=1e-12, estimate_kappa=True)
    finally:
        g.close()
    et = oop.prepare_source(scheme, eta)
    mask, _ = oop.solve_subspace(scheme)
    if mask is None:
        A = lambda v: oop.prec(scheme, v)
        Ad = lambda v: oop.prec_dag(scheme, v)
    else:
        A = lambda v: mask * oop.prec(scheme, mask * v)
        Ad = lambda v: mask * oop.prec_dag(scheme, mask * v)
        et = mask * et
    _, oi = krylov.cgnr(A, Ad, et, 1e-12)
    lmin, lmax, kap = krylov.lanczos_kappa(oi["alphas"], oi["betas"])
    assert abs(info["kappa_est"] / kap - 1) < 0.01, (scheme, info["kappa_est"], kap)
    assert abs(info["lambda_max"] / lmax - 1) < 0.01 and abs(info["lambda_min"] / lmin - 1) < 0.01


@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
def test_cutoff_trick(case, prec):
    """The cutoff trick (tp_op_set_cutoff, Sec. II.A eq:cutoff) with a threshold that drops
    about half of every line's Woodbury corrections: T^-1, T^dagger^-1, C_L, C_R and the
    TEMPORAL_SCHUR apply, S_L and S_R against the oracle's cutoff variant (the App. B sequence
    for clover, eq:TPrecFull for Wilson, built from the cut C_L and C_R); the cut operator
    differs from the exact one.  A mixed solve with the production threshold (the FP32 unit
    roundoff 2^-24) still reaches 1e-10; the half-line threshold drops terms of order 0.1, too
    coarse for a consistent preconditioner."""
    from oracle.temporal import cutoff_slices
    o, g = case["oop"], case["gop"]
    lt = case["dims"][3]
    mu = o.mu
    # 1.5x the bound at mid-line (no slice sits on the threshold: ln 1.5 / ln mu is not an
    # integer), at least 1e-6 so that the dropped terms show in FP64 on long lines too
    eps = max(1.5 * np.sqrt(3) * mu ** (-(lt // 2)), 1e-6)
    oc = OOp(case["U"], case["m0"], case["xi"], float(case["bc"]), o.c_s, o.c_t, eps)
    e, te = case["eta"], case["teta"]
    try:
        dropped = g.set_cutoff(eps)
        assert dropped == int(cutoff_slices(lt, mu, eps).sum()) == int(cutoff_slices(lt, mu, eps, True).sum())
        assert 0 < dropped < lt
        t0, t1 = TOL[prec]
        _close(_np(g.apply_Tinv(te, prec)), oc.tmp.Tinv(e), t0, "cut T^-1")
        _close(_np(g.apply_Tinv(te, prec, dagger=True)), oc.tmp.Tdaginv(e), t0, "cut T^dag^-1")
        _close(_np(g.apply_CL(te, prec)), oc.tmp.CL(e), t0, "cut C_L")
        _close(_np(g.apply_CR(te, prec)), oc.tmp.CR(e), t0, "cut C_R")
        want = oc.tschur_ilu_sequence(e) if o.clover else oc.tschur_closed_form(e)
        got = _np(g.apply_prec(te, "TEMPORAL_SCHUR", prec))
        _close(got, want, t1, "cut TEMPORAL_SCHUR")
        _close(_np(g.prepare_source(te, "TEMPORAL_SCHUR", prec)), oc.tschur_SL(e), t1, "cut S_L")
        _close(_np(g.reconstruct(te, "TEMPORAL_SCHUR", prec)), oc.tschur_SR(e), t1, "cut S_R")
        if prec == "F64":
            assert _rel(got, o.tschur_ilu_sequence(e) if o.clover else o.tschur_closed_form(e)) > 1e-12
        else:
            g.set_cutoff(2.0 ** -24)
            x, info = g.solve(te, scheme="TEMPORAL_SCHUR", prec=prec, tol=1e-10)
            true = np.linalg.norm(e - o.M(_np(x))) / np.linalg.norm(e)
            assert true <= 1.05e-10, (info, true)
    finally:
        assert g.set_cutoff(0.0) == 0
