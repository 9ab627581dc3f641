"""The oracle evaluated at a few sites or time lines of a lattice too large for it.

Test infrastructure only (see the package header).  Nothing here restates the
method: every value comes from the full-lattice functions of `wilson` and
`temporal`, called on a small piece of the lattice that holds everything the
sampled output depends on.

* M psi at a site x depends on psi at x and its eight neighbours, on the links
  leaving x and arriving at x, and on the clover leaves at x, which stay within
  one step in each of two directions (Sec. II, the SW term).  So the oracle's M
  on the periodic 3^4 window centred on x gives the exact value at the centre.
  The time-boundary phase b of the fermion field is put on the window's copies
  of psi that crossed the boundary (the window's own wrap is never used by the
  centre); the clover is built from closed loops and carries no phase.
* T^-1 and T^dagger^-1 act on each time line separately (Sec. II.A), so the
  oracle applied to a lattice of one spatial site, holding one line's links
  and spinor, is exact for that line.
* (A + mu - D_t)^-1 also acts on each time line separately, but A on the line
  depends on the links one step away in two spatial directions; the oracle's
  operator on the periodic 3x3x3 spatial window around the line, of full time
  extent, has the exact clover term on the centre line, and its inverse there
  is the lattice's.
"""
import numpy as np

from . import temporal as T
from . import wilson as W
from .schemes import Operator


def _window_index(c, n):
    return [(c - 1) % n, c, (c + 1) % n]


def M_at_sites(U, psi, sites, m0, gamma_f, b=-1.0, c_s=0.0, c_t=0.0, dagger=False):
    """(M psi)(x) for each x = (x, y, z, t) in `sites`; returns [n, 4, 3].

    U: [4][Lt][Lz][Ly][Lx][3][3], psi: [Lt][Lz][Ly][Lx][4][3] (canonical order)."""
    lt, lz, ly, lx = psi.shape[:4]
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    for n, (x, y, z, t) in enumerate(sites):
        it, iz, iy, ix = (_window_index(t, lt), _window_index(z, lz), _window_index(y, ly),
                          _window_index(x, lx))
        sel = np.ix_(it, iz, iy, ix)
        Uw = np.stack([U[mu][sel] for mu in range(4)])
        pw = psi[sel].copy()
        # phase of the copies that crossed the time boundary relative to the centre
        if t == lt - 1:
            pw[2] *= b
        if t == 0:
            pw[0] *= b
        A = W.clover_field(Uw, c_s, c_t) if (c_s != 0.0 or c_t != 0.0) else None
        f = W.apply_Mdag if dagger else W.apply_M
        out[n] = f(Uw, pw, m0, gamma_f, 1.0, A)[1, 1, 1, 1]
    return out


def Tinv_on_lines(U, psi, lines, mu, b=-1.0, dagger=False, eps=0.0):
    """T^-1 (or T^dagger^-1) psi on the time lines (x, y, z) in `lines`; returns [n, Lt, 4, 3].
    eps > 0: with the cutoff trick of eq:cutoff at that threshold."""
    out = []
    for (x, y, z) in lines:
        ut = U[3][:, z, y, x][:, None, None, None]
        p = psi[:, z, y, x][:, None, None, None]
        f = T.apply_Tdaginv if dagger else T.apply_Tinv
        out.append(f(ut, p, mu, b, eps=eps)[:, 0, 0, 0])
    return np.stack(out)


def sw_temporal_inv_on_lines(U, psi, lines, m0, gamma_f, b=-1.0, c_s=0.0, c_t=0.0):
    """(A + mu - D_t)^-1 psi on the time lines (x, y, z) in `lines`, the left factor of full
    SW temporal preconditioning; returns [n, Lt, 4, 3]."""
    lt, lz, ly, lx = psi.shape[:4]
    if min(lx, ly, lz) < 3:
        raise ValueError("spatial extents of at least 3 are needed for the window")
    out = []
    for (x, y, z) in lines:
        sel = np.ix_(range(lt), _window_index(z, lz), _window_index(y, ly), _window_index(x, lx))
        Uw = np.stack([U[mu][sel] for mu in range(4)])
        op = Operator(Uw, m0, gamma_f, b, c_s, c_t)
        out.append(op.T_inv(psi[sel].copy())[:, 1, 1, 1])
    return np.stack(out)
