"""Fields in the library's own layouts (tp_field): conversions, applies, source preparation and
reconstruction on internal fields against the canonical-in/canonical-out entry points (the
same kernels, so the results agree to the last bit), one-parity fields, batches, refusals, and
the paper's flow (Sec. II.A-B: set-up once, S_L eta, Krylov on Mt, x = S_R y) driven by a
BiCGStab written here in torch on F64 internal fields, checked with the oracle's M."""
import numpy as np
import pytest
import torch

import synth
from oracle.schemes import Operator as OOp

pytestmark = pytest.mark.gpu

CASES = {
    "clover_8x16": ((8, 4, 4, 16), 0.35, 0.12, 3.0, -0.05, 1.6, 1.0),
    "wilson_4x8": ((4, 4, 2, 8), 0.3, 0.1, 3.0, -0.05, 0.0, 0.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_0910_0992_amd import Operator
    dims, es, et, xi, m0, cs, ct = CASES[request.param]
    U = synth.make_links(dims, es, et, 1000)
    g = Operator(torch.from_numpy(U).cuda(), m0, xi, cs / xi, ct, -1)
    eta = torch.from_numpy(synth.make_source(dims, 2000)).cuda()
    print(f"[fields] {request.param} dims={dims}", flush=True)
    yield dict(name=request.param, dims=dims, U=U, g=g, eta=eta, xi=xi, m0=m0, cs=cs / xi, ct=ct,
               clover=cs != 0.0)
    g.close()


def _parity(dims, four_d):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    p = (x + y + z + (t if four_d else 0)) % 2
    return torch.from_numpy(p.astype(np.float64)[..., None, None]).cuda()


@pytest.mark.parametrize("layout", ["P3", "P4"])
@pytest.mark.parametrize("prec", ["F64", "F32", "F16N"])
def test_round_trip_and_subsets(case, layout, prec):
    g, eta = case["g"], case["eta"]
    tol = {"F64": 1e-15, "F32": 1e-7, "F16N": 1e-3}[prec]
    back = g.from_field(g.to_field(eta, layout, prec))[0]
    assert (torch.linalg.vector_norm(back - eta) / torch.linalg.vector_norm(eta)).item() < tol
    odd = _parity(case["dims"], layout == "P4")
    for subset, mask in (("EVEN", 1 - odd), ("ODD", odd)):
        f = g.to_field(eta, layout, prec, subset)
        assert f.buf.numel() == g.field_bytes(layout, prec, subset) < g.field_bytes(layout, prec)
        back = g.from_field(f)[0]
        assert torch.count_nonzero(back * (1 - mask)) == 0
        ref = eta * mask
        assert (torch.linalg.vector_norm(back - ref) / torch.linalg.vector_norm(ref)).item() < tol
        # one parity into a FULL field: the other parity is zero
        full = g.convert_field(g.field(layout, prec), f)
        assert torch.equal(g.from_field(full), g.from_field(f))


@pytest.mark.parametrize("scheme,prec", [("TEMPORAL_SCHUR", "F16N"), ("TEMPORAL_SCHUR", "F64"),
                                         ("TEMPORAL", "F32"), ("UNPREC", "F64"), ("SCHUR4D", "F32"),
                                         ("TEMPORAL_SCHUR3D", "F64"), ("TEMPORAL_FULLSW", "F32")])
def test_field_applies_match_canonical_entry_points(case, scheme, prec):
    g, eta = case["g"], case["eta"]
    lay = "P4" if scheme == "SCHUR4D" else "P3"
    f = g.to_field(eta, lay, prec)
    for dagger in (False, True):
        assert torch.equal(g.from_field(g.apply_prec_field(f, scheme, dagger))[0],
                           g.apply_prec(eta, scheme, prec, dagger=dagger))
    et = g.prepare_source_field(eta, scheme, prec)
    assert torch.equal(g.from_field(et)[0], g.prepare_source(eta, scheme, prec))
    assert torch.equal(g.prepare_source_field(f, scheme, prec).buf, et.buf)
    assert torch.equal(g.reconstruct_field(f, scheme)[0], g.reconstruct(eta, scheme, prec))
    # odd-block schemes: the ODD field apply is the odd part of the FULL apply
    sub = scheme in ("SCHUR4D", "TEMPORAL_SCHUR3D") or (scheme == "TEMPORAL_SCHUR" and not case["clover"])
    fo = g.to_field(eta, lay, prec, "ODD")
    if sub:
        yo = g.apply_prec_field(fo, scheme)
        yf = g.apply_prec_field(f, scheme)
        assert torch.equal(yo.buf, g.convert_field(g.field(lay, prec, "ODD"), yf).buf)
    else:
        from paper_0910_0992_amd._lib import TprecError
        with pytest.raises(TprecError, match="odd block"):
            g.apply_prec_field(fo, scheme)


def test_batched_fields(case):
    g, eta = case["g"], case["eta"]
    e2 = torch.from_numpy(synth.make_source(case["dims"], 2001)).cuda()
    f = g.to_field(torch.stack([eta, e2]), "P3", "F16N")
    y = g.from_field(g.apply_prec_field(f, "TEMPORAL_SCHUR"))
    for k, e in enumerate((eta, e2)):
        assert torch.equal(y[k], g.apply_prec(e, "TEMPORAL_SCHUR", "F16N"))


def test_field_refusals(case):
    from paper_0910_0992_amd._lib import TprecError
    g, eta = case["g"], case["eta"]
    f3, f4 = g.to_field(eta, "P3"), g.to_field(eta, "P4")
    with pytest.raises(TprecError, match="layout"):
        g.apply_prec_field(f4, "TEMPORAL_SCHUR")
    with pytest.raises(TprecError, match="internal layouts differ"):
        g.convert_field(f4, f3)
    with pytest.raises(TprecError, match="FULL or ODD"):
        g.apply_prec_field(g.to_field(eta, "P3", "F64", "EVEN"), "TEMPORAL_SCHUR")


def _bicgstab(A, b, tol, maxit=5000):
    """Textbook BiCGStab (van der Vorst 1992) on complex vectors, from x = 0."""
    x = torch.zeros_like(b)
    r = b.clone()
    rh = b.clone()
    p = r.clone()
    rho = torch.vdot(rh, r)
    bn = torch.linalg.vector_norm(b)
    for it in range(maxit):
        v = A(p)
        al = rho / torch.vdot(rh, v)
        s = r - al * v
        t = A(s)
        om = torch.vdot(t, s) / torch.vdot(t, t)
        x = x + al * p + om * s
        r = s - om * t
        if torch.linalg.vector_norm(r) <= tol * bn:
            return x, it + 1
        rn = torch.vdot(rh, r)
        p = r + (rn / rho) * (al / om) * (p - om * v)
        rho = rn
    raise RuntimeError("no convergence")


@pytest.mark.parametrize("scheme", ["TEMPORAL_SCHUR", "TEMPORAL_SCHUR3D", "TEMPORAL_FULLSW"])
def test_external_krylov_on_internal_fields(case, scheme):
    """A solver outside the library: eta~ = S_L eta once, BiCGStab on Mt with the library's
    applies on F64 internal fields (the odd block for odd-block schemes, held in ODD fields),
    x = S_R y; the oracle's M gives the true residual."""
    g, eta = case["g"], case["eta"]
    oop = OOp(case["U"], case["m0"], case["xi"], -1.0, case["cs"], case["ct"])
    et = g.prepare_source_field(eta, scheme)
    sub = scheme == "TEMPORAL_SCHUR3D" or (scheme == "TEMPORAL_SCHUR" and not case["clover"])
    if sub:
        eo = g.convert_field(g.field("P3", "F64", "ODD"), et)
        work = g.field("P3", "F64", "ODD")
        vec = lambda f: f.buf.view(torch.complex128)

        def A(v):
            work.buf.view(torch.complex128).copy_(v)
            return vec(g.apply_prec_field(work, scheme)).clone()
        yo, its = _bicgstab(A, vec(eo).clone(), 1e-12)
        work.buf.view(torch.complex128).copy_(yo)
        y = g.convert_field(g.field("P3", "F64"), work)
        # even part of y: eta~_e (the even block of Mt is the identity)
        ye = g.convert_field(g.field("P3", "F64", "EVEN"), et)
        both = g.from_field(y)[0] + g.from_field(ye)[0]
        y = g.to_field(both, "P3", "F64")
    else:
        work = g.field("P3", "F64")

        def A(v):
            work.as_complex()[0].copy_(v)
            return g.apply_prec_field(work, scheme).as_complex()[0].clone()
        yv, its = _bicgstab(A, et.as_complex()[0].clone(), 1e-12)
        work.as_complex()[0].copy_(yv)
        y = work
    x = g.reconstruct_field(y, scheme)[0].cpu().numpy()
    e = eta.cpu().numpy()
    true = np.linalg.norm(e - oop.M(x)) / np.linalg.norm(e)
    print(f"[fields] external BiCGStab {scheme}: {its} iterations, true residual {true:.2e}", flush=True)
    assert true <= 1.05e-10


@pytest.mark.gpu
def test_operator_left_open_at_exit():
    """An operator that is never closed is released at interpreter exit through the torch
    allocator without errors (its memory callbacks must not outlive torch's teardown)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import torch, synth\n"
            "from paper_0910_0992_amd import Operator\n"
            "U = synth.make_links((4, 4, 4, 8), 0.3, 0.1, 1000)\n"
            "op = Operator(torch.from_numpy(U).cuda(), -0.05, 3.0, 0.5, 1.0, -1)\n"
            "eta = torch.from_numpy(synth.make_source((4, 4, 4, 8), 2000)).cuda()\n"
            "x, info = op.solve(eta, scheme='TEMPORAL_SCHUR', prec='F32', tol=1e-8)\n"
            "print('solved', info['iters'], flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                       cwd=root, env=dict(os.environ, PYTHONPATH=root))
    assert r.returncode == 0, r.stderr[-2000:]
    assert "solved" in r.stdout
    assert "Exception ignored" not in r.stderr and "Traceback" not in r.stderr, r.stderr[-2000:]
