"""tp_apply_prec_noalloc, the apply for callers that cannot allocate: through the C ABI, against
tp_apply_prec on the same inputs (the same kernels, so the results agree to the last bit), on
two calls in a row with the second on a smaller lattice, without any device allocation during
the call (the binding hands all of the library's device memory to torch's caching allocator,
so torch's count and the library's own count must not move), and the documented refusals."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _op(dims, clover=True):
    from paper_0910_0992_amd import Operator
    U = synth.make_links(dims, 0.35, 0.12, 1000)
    xi = 3.5
    cs, ct = (1.6 / xi, 1.0) if clover else (0.0, 0.0)
    return Operator(torch.from_numpy(U).cuda(), -0.05, xi, cs, ct, -1)


def _noalloc(op, psi, scheme, prec, dagger=False):
    from paper_0910_0992_amd import _lib as L
    from paper_0910_0992_amd.api import _prec, _scheme
    out = torch.empty_like(psi)
    torch.cuda.synchronize()
    before = (op.device_bytes(), torch.cuda.memory_allocated())
    op._bind_stream()
    st = op._lib.tp_apply_prec_noalloc(op._op, _scheme(scheme), _prec(prec), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(psi.data_ptr()), int(dagger))
    L.check(st)
    torch.cuda.synchronize()
    after = (op.device_bytes(), torch.cuda.memory_allocated())
    assert before == after, (before, after)
    return out


CALLS = [("TEMPORAL_SCHUR", "F16N", False), ("TEMPORAL_SCHUR", "F32", True), ("TEMPORAL_SCHUR", "F64", False),
         ("SCHUR4D", "F64", True), ("TEMPORAL", "F32", False), ("UNPREC", "F64", True)]


@pytest.mark.parametrize("clover", [True, False])
def test_noalloc_matches_apply_prec(clover):
    """Two calls in a row, the second on a smaller lattice: each bit-identical to tp_apply_prec."""
    for dims in [(8, 8, 8, 32), (4, 2, 2, 12)]:
        print(f"[noalloc] dims={dims} clover={clover}", flush=True)
        op = _op(dims, clover)
        try:
            psi = torch.from_numpy(synth.make_source(dims, 2000)).cuda()
            got = [_noalloc(op, psi, s, p, d) for s, p, d in CALLS]  # before any allocating apply
            for (s, p, d), y in zip(CALLS, got):
                ref = op.apply_prec(psi, s, p, dagger=d)
                assert torch.equal(y, ref), (dims, s, p, d)
            # after the allocating applies, and again (the scratch keeps the last call's data)
            y2 = _noalloc(op, psi, "TEMPORAL_SCHUR", "F16N")
            assert torch.equal(y2, op.apply_prec(psi, "TEMPORAL_SCHUR", "F16N"))
        finally:
            op.close()


@pytest.mark.parametrize("scheme,prec", [("TEMPORAL_SCHUR3D", "F64"), ("TEMPORAL_FULLSW", "F32")])
def test_noalloc_block_lu_after_factorisation(scheme, prec):
    """The block-LU schemes are refused until an allocating apply has built their factors,
    then match it, both ways round."""
    dims = (6, 4, 4, 16)
    op = _op(dims)
    try:
        psi = torch.from_numpy(synth.make_source(dims, 2001)).cuda()
        from paper_0910_0992_amd._lib import TprecError
        with pytest.raises(TprecError, match="factors"):
            _noalloc(op, psi, scheme, prec)
        ref = op.apply_prec(psi, scheme, prec)  # builds the factors
        assert torch.equal(_noalloc(op, psi, scheme, prec), ref)
        assert torch.equal(_noalloc(op, psi, scheme, prec, True), op.apply_prec(psi, scheme, prec, dagger=True))
    finally:
        op.close()


def test_noalloc_refuses_lattices_beyond_the_scratch():
    """16^3x32 in FP64 needs 6 fields of 24 MiB for TEMPORAL_SCHUR: more than 64 MiB."""
    from paper_0910_0992_amd._lib import TprecError
    dims = (16, 16, 16, 32)
    op = _op(dims)
    try:
        psi = torch.from_numpy(synth.make_source(dims, 2002)).cuda()
        with pytest.raises(TprecError, match="scratch"):
            _noalloc(op, psi, "TEMPORAL_SCHUR", "F64")
        # F16N fits (6 fields of 7 MiB) and matches
        y = _noalloc(op, psi, "TEMPORAL_SCHUR", "F16N")
        assert torch.equal(y, op.apply_prec(psi, "TEMPORAL_SCHUR", "F16N"))
    finally:
        op.close()
