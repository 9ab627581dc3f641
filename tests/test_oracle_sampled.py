"""The sampled oracle (M at single sites, T^-1 and (A + mu - D_t)^-1 on single time lines) against the
full-lattice oracle at every kind of site: interior, spatial edges, both time
boundaries, periodic and antiperiodic, Wilson and clover, and lattices with an
extent of 2 (where both neighbours in a direction are the same site)."""
import numpy as np
import pytest

import synth
from oracle import sampled, temporal as T, wilson as W

CASES = [((4, 4, 4, 8), -1.0, 1.2, 0.9), ((6, 4, 2, 6), -1.0, 0.0, 0.0),
         ((4, 2, 4, 4), 1.0, 1.6, 1.0), ((2, 2, 2, 5), -1.0, 0.7, 1.3)]


def _sites(dims, rng, n=12):
    lx, ly, lz, lt = dims
    fixed = [(0, 0, 0, 0), (lx - 1, ly - 1, lz - 1, lt - 1), (0, ly - 1, 1 % lz, lt - 1),
             (lx - 1, 0, lz - 1, 0), (1, 1, 1, lt // 2)]
    rnd = [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(n)]
    return fixed + rnd


@pytest.mark.parametrize("dims,b,c_s,c_t", CASES)
@pytest.mark.parametrize("dagger", [False, True])
def test_M_at_sites_matches_full_lattice(dims, b, c_s, c_t, dagger):
    U = synth.make_links(dims, 0.5, 0.3, 11)
    psi = synth.make_source(dims, 12)
    m0, gf = -0.05, 2.5
    A = W.clover_field(U, c_s, c_t) if c_s or c_t else None
    full = (W.apply_Mdag if dagger else W.apply_M)(U, psi, m0, gf, b, A)
    sites = _sites(dims, np.random.default_rng(5))
    got = sampled.M_at_sites(U, psi, sites, m0, gf, b, c_s, c_t, dagger=dagger)
    ref = np.stack([full[t, z, y, x] for (x, y, z, t) in sites])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dims,b", [((4, 4, 2, 8), -1.0), ((2, 4, 2, 7), 1.0)])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_Tinv_on_lines_matches_full_lattice(dims, b, dagger, eps):
    U = synth.make_links(dims, 0.5, 0.3, 13)
    psi = synth.make_source(dims, 14)
    mu = 1.7
    full = (T.apply_Tdaginv if dagger else T.apply_Tinv)(U[3], psi, mu, b, eps=eps)
    lines = [(0, 0, 0), (dims[0] - 1, dims[1] - 1, dims[2] - 1), (1, 2 % dims[1], 1)]
    got = sampled.Tinv_on_lines(U, psi, lines, mu, b, dagger=dagger, eps=eps)
    ref = np.stack([full[:, z, y, x] for (x, y, z) in lines])
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dims,b,c_s,c_t", [((4, 6, 4, 8), -1.0, 1.2, 0.9), ((6, 4, 4, 5), 1.0, 0.0, 0.0)])
def test_sw_temporal_inv_on_lines_matches_full_lattice(dims, b, c_s, c_t):
    """(A + mu - D_t)^-1 on single lines from the 3x3x3 window against the full lattice's
    inverse, on lines at the spatial edges (the window wraps) and inside."""
    from oracle.schemes import Operator
    U = synth.make_links(dims, 0.5, 0.3, 15)
    psi = synth.make_source(dims, 16)
    m0, gf = -0.05, 2.5
    full = Operator(U, m0, gf, b, c_s, c_t).T_inv(psi)
    lines = [(0, 0, 0), (dims[0] - 1, dims[1] - 1, dims[2] - 1), (1, 2, 3), (2, 5 % dims[1], 0)]
    got = sampled.sw_temporal_inv_on_lines(U, psi, lines, m0, gf, b, c_s, c_t)
    ref = np.stack([full[:, z, y, x] for (x, y, z) in lines])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
