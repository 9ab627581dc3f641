"""Pins of the oracle's gradient against central finite differences with exact
(dense LU) solves, so that the only error is the O(h^2) truncation."""
import numpy as np
import pytest

import synth
from oracle import force
from oracle.schemes import Operator

DIMS = (2, 2, 4, 4)


def _expi(h):
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def _loss_dense(U, eta, m0, gf, b, A):
    op = Operator(U, m0, gf, b)
    op.A, op.clover = A, A is not None
    lx, ly, lz, lt = DIMS
    n = lx * ly * lz * lt * 12
    M = np.array([op.M(np.eye(n)[k].reshape(lt, lz, ly, lx, 4, 3)).ravel() for k in range(n)]).T
    x = np.linalg.solve(M, eta.ravel())
    return float(np.vdot(x, x).real)


@pytest.mark.parametrize("cs,ct", [(0.0, 0.0), (1.6 / 3.0, 1.0)])
def test_link_and_source_gradient_vs_fd(cs, ct):
    U = synth.make_links(DIMS, 0.5, 0.3, 1000)
    eta = synth.make_source(DIMS, 2000)
    op = Operator(U, -0.05, 3.0, -1.0, cs, ct)
    L, lam, grad_U, G, x = force.loss_and_grads(op, eta, "TEMPORAL_SCHUR", 1e-14)
    A = op.A
    assert np.isclose(L, _loss_dense(U, eta, -0.05, 3.0, -1.0, A), rtol=1e-12)
    h = 1e-5
    for k in range(3):
        om = synth.make_algebra_field(DIMS, 4000 + k)
        Lp = _loss_dense(_expi(h * om) @ U, eta, -0.05, 3.0, -1.0, A)
        Lm = _loss_dense(_expi(-h * om) @ U, eta, -0.05, 3.0, -1.0, A)
        fd = (Lp - Lm) / (2 * h)
        an = np.sum(np.einsum("...ij,...ji->...", om, G)).real
        assert abs(fd - an) < 1e-7 * abs(L), (fd, an)
        # the raw Wirtinger gradient gives the same derivative for dU = i omega U
        an2 = np.vdot(grad_U, 1j * om @ U).real
        assert abs(an2 - an) < 1e-10 * abs(an)
    # source gradient: the loss is quadratic in eta
    d = synth.make_source(DIMS, 2001)
    Lp = _loss_dense(U, eta + h * d, -0.05, 3.0, -1.0, A)
    Lm = _loss_dense(U, eta - h * d, -0.05, 3.0, -1.0, A)
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - np.vdot(lam, d).real) < 1e-7 * abs(L)


def test_force_is_traceless_hermitian():
    U = synth.make_links(DIMS, 0.5, 0.3, 1001)
    eta = synth.make_source(DIMS, 2002)
    op = Operator(U, -0.05, 3.0, -1.0)
    _, _, _, G, _ = force.loss_and_grads(op, eta, "UNPREC", 1e-13)
    assert np.abs(G - np.conj(np.swapaxes(G, -1, -2))).max() < 1e-14 * np.abs(G).max()
    assert np.abs(np.trace(G, axis1=-2, axis2=-1)).max() < 1e-13 * np.abs(G).max()


def test_torch_clover_matches_clover_field():
    """The differentiable transcription of the SW term equals wilson.clover_field."""
    import torch
    U = synth.make_links(DIMS, 0.5, 0.3, 1002)
    got = force._torch_clover(torch.from_numpy(U), 0.7, 1.3).numpy()
    from oracle import wilson as W
    ref = W.clover_field(U, 0.7, 1.3)
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("b", [-1.0, 1.0])
def test_full_link_gradient_vs_fd_with_clover(b):
    """With A = A(U) recomputed for every perturbed field, central differences of
    |M^-1 eta|^2 (exact dense solves) match the hopping plus SW-term gradient; the
    hopping part alone misses the difference."""
    from oracle import wilson as W
    cs, ct = 1.6 / 3.0, 1.0
    U = synth.make_links(DIMS, 0.5, 0.3, 1003)
    eta = synth.make_source(DIMS, 2003)
    op = Operator(U, -0.05, 3.0, b, cs, ct)
    L, lam, _, _, x = force.loss_and_grads(op, eta, "TEMPORAL_SCHUR", 1e-14)
    g_full, G_full = force.full_link_gradient(op, x, lam)
    g_hop, _ = force.link_gradient(op, x, lam)
    h = 1e-5
    for k in range(3):
        om = synth.make_algebra_field(DIMS, 4010 + k)
        Up, Um = _expi(h * om) @ U, _expi(-h * om) @ U
        Lp = _loss_dense(Up, eta, -0.05, 3.0, b, W.clover_field(Up, cs, ct))
        Lm = _loss_dense(Um, eta, -0.05, 3.0, b, W.clover_field(Um, cs, ct))
        fd = (Lp - Lm) / (2 * h)
        an = np.vdot(g_full, 1j * om @ U).real
        assert abs(fd - an) < 1e-7 * abs(L), (fd, an)
        assert np.isclose(np.sum(np.einsum("...ij,...ji->...", om, G_full)).real, an, rtol=1e-10)
        hop_only = np.vdot(g_hop, 1j * om @ U).real
        assert abs(fd - hop_only) > 1e3 * abs(fd - an)
