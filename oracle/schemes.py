"""The fermion operator and its four preconditioning schemes (Sec. II.A, II.B).

Every scheme writes M = S_L^-1  Mt  S_R^-1 and solves
    eta~ = S_L eta,   Mt y = eta~,   x = S_R y.

UNPREC          S_L = S_R = 1, Mt = M.
SCHUR4D         4D parity p4 = (-1)^(x+y+z+t).  LDU factorisation of Sec. II.B:
                M^ee = A + mu, M^eo = -D_w^eo, D_w = D_s/gamma_f + D_t;
                S_L = L^-1, S_R = U^-1 and Mt = diag(M^ee, M^oo - M^oe (M^ee)^-1 M^eo).
TEMPORAL        S_L = C_L, S_R = C_R, Mt = C_L M C_R (Sec. II.A).
TEMPORAL_SCHUR  3D parity p3 = (-1)^(x+y+z); M^ee = A + mu - D_t on even sites,
                M^eo = -D_s^eo/gamma_f.  S_L and S_R are the block-triangular
                matrices of Sec. II.B; Mt3 = S_L M S_R.  For Wilson fermions this
                is eq:TPrecFull; for clover with the Wilson C_L, C_R ("partial SW
                temporal preconditioning") it is eq:TPrecPartial, the 3D ILU scheme.
TEMPORAL_SCHUR3D  the same p3 blocks with the even block inverted exactly (temporal
                preconditioning combined with 3D-Schur, Sec. II.B and App. A):
                S_o = M^oo - M^oe (M^ee)^-1 M^eo and Mt = diag(1, C_L^o S_o C_R^o),
                S_L = diag((M^ee)^-1, C_L^o) L^-1, S_R = U^-1 diag(1, C_R^o).  Here
                (M^ee)^-1 is a sparse direct solve of the assembled even block;
                for Wilson fermions M^ee = mu - D_t = (C_R C_L)^-1 and the scheme is
                eq:TPrecFull again.
TEMPORAL_FULLSW full SW temporal preconditioning on the whole lattice (Sec. II.A, App. A):
                with T = A + mu - D_t inverted exactly, C_L = T^-1 and C_R = 1, so
                Q-bar = C_L T C_R = 1 and Mt = C_L M C_R = 1 - T^-1 D_s / gamma_f,
                S_L = T^-1, S_R = 1.  Mt is not gamma5-hermitian: its adjoint is
                gamma5 (1 - D_s T^-1 / gamma_f) gamma5.

Blocks are formed literally: K^{ab} psi = mask_a * K(mask_b * psi) on the full
lattice, so every identity below can be checked by eye against the paper.

The printed S_L^-1, S_R^-1 of Sec. II.B are not the inverses of S_L, S_R (their
triangularity is swapped); they are not needed, because the solution is
recovered as x = S_R y.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dirac import GAMMA5, PT_MINUS, PT_PLUS, spin_apply
from . import wilson as W
from .temporal import Temporal

SCHEMES = ("UNPREC", "SCHUR4D", "TEMPORAL", "TEMPORAL_SCHUR", "TEMPORAL_SCHUR3D", "TEMPORAL_FULLSW")


def parity_masks(dims, four_d: bool):
    """(even, odd) masks shaped [Lt,Lz,Ly,Lx,1,1]; p3 uses x+y+z, p4 adds t."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    p = (x + y + z + (t if four_d else 0)) % 2
    even = (p == 0).astype(np.float64)[..., None, None]
    return even, 1.0 - even


class Operator:
    """M = A + mu - D_t - D_s/gamma_f bound to links, mass, anisotropy, clover and BC."""

    def __init__(self, U, m0, gamma_f, b=-1.0, c_s=0.0, c_t=0.0, cutoff_eps=0.0):
        self.U = U
        self.m0 = m0
        self.gamma_f = gamma_f
        self.b = b
        self.c_s, self.c_t = c_s, c_t
        self.mu = W.mass_term(m0, gamma_f)
        self.dims = (U.shape[4], U.shape[3], U.shape[2], U.shape[1])
        self.clover = (c_s != 0.0) or (c_t != 0.0)
        self.A = W.clover_field(U, c_s, c_t) if self.clover else None
        # cutoff_eps > 0: the cutoff trick in every T^-1 and T^dagger^-1 (C_L, C_R, and so the
        # App. B sequence, S_L and S_R of TEMPORAL_SCHUR built from them)
        self.tmp = Temporal(U, self.mu, b, cutoff_eps)
        self.e3, self.o3 = parity_masks(self.dims, False)
        self.e4, self.o4 = parity_masks(self.dims, True)
        self._Amu_inv = None
        self._mee = None

    # ---- the unpreconditioned pieces -------------------------------------------------
    def M(self, psi):
        return W.apply_M(self.U, psi, self.m0, self.gamma_f, self.b, self.A)

    def Mdag(self, psi):
        return W.apply_Mdag(self.U, psi, self.m0, self.gamma_f, self.b, self.A)

    def Ds(self, psi):
        return W.hop_s(self.U, psi, self.b)

    def Dt(self, psi):
        return W.hop_t(self.U, psi, self.b)

    def Aop(self, psi):
        return W.apply_A(self.A, psi) if self.clover else np.zeros_like(psi)

    def Amu(self, psi):
        """(A + mu) psi."""
        return self.Aop(psi) + self.mu * psi

    def Amu_inv(self, psi):
        """(A + mu)^-1 psi, site by site."""
        if self._Amu_inv is None:
            a = self.A if self.clover else np.zeros(tuple(reversed(self.dims)) + (12, 12),
                                                    dtype=np.complex128)
            self._Amu_inv = W.clover_plus_mass_inverse(a, self.mu)
        return W.apply_A(self._Amu_inv, psi)

    # ---- 4D Schur (p4) ---------------------------------------------------------------
    def schur4d_Shat(self, psi):
        """M^oo - M^oe (M^ee)^-1 M^eo on the odd p4 sites (blocks cut from M itself)."""
        e, o = self.e4, self.o4
        po = o * psi
        meo = e * self.M(po)
        return o * self.M(po) - o * self.M(e * self.Amu_inv(meo))

    def schur4d(self, psi):
        e, o = self.e4, self.o4
        return e * self.M(e * psi) + self.schur4d_Shat(psi)

    def schur4d_SL(self, eta):
        """L^-1 eta: (eta_e, eta_o - M^oe (M^ee)^-1 eta_e)."""
        e, o = self.e4, self.o4
        return e * eta + o * eta - o * self.M(e * self.Amu_inv(e * eta))

    def schur4d_SR(self, y):
        """U^-1 y: (y_e - (M^ee)^-1 M^eo y_o, y_o)."""
        e, o = self.e4, self.o4
        return e * y - e * self.Amu_inv(e * self.M(o * y)) + o * y

    # ---- temporal --------------------------------------------------------------------
    def temporal(self, psi):
        return self.tmp.CL(self.M(self.tmp.CR(psi)))

    # ---- temporal + 3D Schur / ILU (p3) ----------------------------------------------
    def Dbar_oe(self, psi):
        """D-bar_s^oe = C_L^o D_s^oe C_R^e."""
        return self.tmp.CL(self.o3 * self.Ds(self.tmp.CR(self.e3 * psi)))

    def Dbar_eo(self, psi):
        return self.tmp.CL(self.e3 * self.Ds(self.tmp.CR(self.o3 * psi)))

    def Abar(self, psi):
        """A-bar = C_L A C_R (parity preserving)."""
        return self.tmp.CL(self.Aop(self.tmp.CR(psi)))

    def tschur_SL(self, eta):
        """S_L = [[C_L^e, 0], [D-bar^oe C_L^e / gamma_f, C_L^o]]."""
        e, o, g = self.e3, self.o3, self.gamma_f
        cle = self.tmp.CL(e * eta)
        return cle + self.Dbar_oe(cle) / g + self.tmp.CL(o * eta)

    def tschur_SR(self, y):
        """S_R = [[C_R^e, C_R^e D-bar^eo / gamma_f], [0, C_R^o]]."""
        e, o, g = self.e3, self.o3, self.gamma_f
        return self.tmp.CR(e * y) + self.tmp.CR(self.Dbar_eo(y)) / g + self.tmp.CR(o * y)

    def tschur(self, psi):
        """Mt3 = S_L M S_R, literally."""
        return self.tschur_SL(self.M(self.tschur_SR(psi)))

    def tschur_closed_form(self, psi):
        """eq:TPrecPartial (reduces to eq:TPrecFull when A = 0)."""
        e, o, g = self.e3, self.o3, self.gamma_f
        pe, po = e * psi, o * psi
        db_eo_po = self.Dbar_eo(po)
        out_e = pe + self.Abar(pe) + self.Abar(db_eo_po) / g
        out_o = (self.Dbar_oe(self.Abar(pe)) / g + po + self.Abar(po)
                 - self.Dbar_oe(db_eo_po - self.Abar(db_eo_po)) / g ** 2)
        return e * out_e + o * out_o

    def tschur_ilu_sequence(self, psi):
        """The appendix's six-step sequence for the ILU operator (gamma_f folded into D-bar)."""
        e, o, g = self.e3, self.o3, self.gamma_f
        pe, po = e * psi, o * psi
        t1 = self.Dbar_eo(po) / g
        t2 = self.Abar(t1 + pe)
        chi_e = pe + t2
        chi_o = po + self.Abar(po) + self.Dbar_oe(t2 - t1) / g
        return e * chi_e + o * chi_o

    # ---- temporal + 3D Schur with the exact even block (p3) --------------------------
    def _mee_factor(self, rows=None):
        """Sparse LU of M^ee = A + mu - D_t on the even p3 sites (identity on odd sites), or on
        the sites where `rows` is true (all sites: the whole-lattice T = A + mu - D_t).

        Assembled from the definitions (Sec. II.B; D_t of Sec. II.A with the boundary phase b
        on the wrapping hops): diagonal blocks A(x) + mu, and the temporal hops
        -P_- (x) U_t(x) to t+1 and -P_+ (x) U_t(x - t)^dagger to t-1, index spin*3 + colour.
        M^ee keeps the spatial site, so the matrix is block diagonal over time lines."""
        lx, ly, lz, lt = self.dims
        n = lx * ly * lz * lt * 12
        idx = np.arange(n).reshape(lt, lz, ly, lx, 12)
        even = (self.e3[..., 0, 0] > 0.5) if rows is None else rows
        diag = np.broadcast_to(self.mu * np.eye(12), (lt, lz, ly, lx, 12, 12)).copy()
        if self.clover:
            diag = diag + self.A
        diag[~even] = np.eye(12)
        ut = self.U[3]
        fwd = -np.einsum("st,...ab->...satb", PT_MINUS, ut).reshape(ut.shape[:4] + (12, 12))
        fwd[-1] *= self.b
        ubk = np.roll(ut, 1, axis=0).conj().swapaxes(-1, -2)
        bwd = -np.einsum("st,...ab->...satb", PT_PLUS, ubk).reshape(ut.shape[:4] + (12, 12))
        bwd[0] *= self.b
        rows, cols, vals = [], [], []
        for blk, col_idx, mask in ((diag, idx, np.ones_like(even)),
                                   (fwd, np.roll(idx, -1, axis=0), even),
                                   (bwd, np.roll(idx, 1, axis=0), even)):
            r = np.broadcast_to(idx[..., :, None], blk.shape)[mask]
            c = np.broadcast_to(col_idx[..., None, :], blk.shape)[mask]
            rows.append(r.ravel())
            cols.append(c.ravel())
            vals.append(blk[mask].ravel())
        m = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n))
        return spla.splu(m)

    def Mee_inv(self, psi):
        """(M^ee)^-1 on the even p3 sites."""
        if self._mee is None:
            self._mee = self._mee_factor()
        out = self._mee.solve(np.ascontiguousarray((self.e3 * psi).ravel()))
        return self.e3 * out.reshape(psi.shape)

    def schur3d_S(self, psi):
        """S_o = M^oo - M^oe (M^ee)^-1 M^eo on the odd p3 sites (blocks cut from M)."""
        e, o = self.e3, self.o3
        po = o * psi
        return o * self.M(po) - o * self.M(e * self.Mee_inv(e * self.M(po)))

    def tschur3d(self, psi):
        """diag(1, C_L^o S_o C_R^o)."""
        e, o = self.e3, self.o3
        return e * psi + o * self.tmp.CL(self.schur3d_S(o * self.tmp.CR(o * psi)))

    def tschur3d_SL(self, eta):
        """((M^ee)^-1 eta_e,  C_L^o [eta_o - M^oe (M^ee)^-1 eta_e])."""
        e, o = self.e3, self.o3
        f = self.Mee_inv(e * eta)
        return f + o * self.tmp.CL(o * eta - o * self.M(f))

    def tschur3d_SR(self, y):
        """(y_e - (M^ee)^-1 M^eo x_o,  x_o = C_R^o y_o)."""
        e, o = self.e3, self.o3
        xo = o * self.tmp.CR(o * y)
        return e * y - self.Mee_inv(e * self.M(xo)) + xo

    # ---- full SW temporal preconditioning on the whole lattice ------------------------
    def T_inv(self, psi):
        """(A + mu - D_t)^-1 on every site (a sparse direct solve of the assembled matrix)."""
        if getattr(self, "_tfull", None) is None:
            lx, ly, lz, lt = self.dims
            self._tfull = self._mee_factor(np.ones((lt, lz, ly, lx), dtype=bool))
        return self._tfull.solve(np.ascontiguousarray(psi.ravel())).reshape(psi.shape)

    def fullsw(self, psi):
        """Mt = 1 - T^-1 D_s / gamma_f."""
        return psi - self.T_inv(self.Ds(psi)) / self.gamma_f

    def fullsw_dag(self, psi):
        """Mt^dagger = 1 - D_s^dagger T^-dagger / gamma_f = gamma5 (1 - D_s T^-1 / gamma_f) gamma5."""
        phi = spin_apply(GAMMA5, psi)
        return spin_apply(GAMMA5, phi - self.Ds(self.T_inv(phi)) / self.gamma_f)

    # ---- scheme dispatch -------------------------------------------------------------
    def prec(self, scheme, psi):
        if scheme == "UNPREC":
            return self.M(psi)
        if scheme == "SCHUR4D":
            return self.schur4d(psi)
        if scheme == "TEMPORAL":
            return self.temporal(psi)
        if scheme == "TEMPORAL_SCHUR":
            return self.tschur(psi)
        if scheme == "TEMPORAL_SCHUR3D":
            return self.tschur3d(psi)
        if scheme == "TEMPORAL_FULLSW":
            return self.fullsw(psi)
        raise ValueError(scheme)

    def prec_dag(self, scheme, psi):
        """Every Mt here but TEMPORAL_FULLSW is gamma5-hermitian, Mt^dagger = gamma5 Mt gamma5."""
        if scheme == "TEMPORAL_FULLSW":
            return self.fullsw_dag(psi)
        return spin_apply(GAMMA5, self.prec(scheme, spin_apply(GAMMA5, psi)))

    def prepare_source(self, scheme, eta):
        if scheme == "UNPREC":
            return eta.copy()
        if scheme == "SCHUR4D":
            return self.schur4d_SL(eta)
        if scheme == "TEMPORAL":
            return self.tmp.CL(eta)
        if scheme == "TEMPORAL_SCHUR":
            return self.tschur_SL(eta)
        if scheme == "TEMPORAL_SCHUR3D":
            return self.tschur3d_SL(eta)
        if scheme == "TEMPORAL_FULLSW":
            return self.T_inv(eta)
        raise ValueError(scheme)

    def reconstruct(self, scheme, y):
        if scheme == "UNPREC":
            return y.copy()
        if scheme == "SCHUR4D":
            return self.schur4d_SR(y)
        if scheme == "TEMPORAL":
            return self.tmp.CR(y)
        if scheme == "TEMPORAL_SCHUR":
            return self.tschur_SR(y)
        if scheme == "TEMPORAL_SCHUR3D":
            return self.tschur3d_SR(y)
        if scheme == "TEMPORAL_FULLSW":
            return y.copy()
        raise ValueError(scheme)

    def solve_subspace(self, scheme):
        """Mask of the sites the Krylov solver works on, and how the rest of y is fixed.

        SCHUR4D: Mt = diag(A+mu, S-hat): y_e = (A+mu)^-1 eta~_e, Krylov on odd p4 sites.
        TEMPORAL_SCHUR, Wilson, and TEMPORAL_SCHUR3D: Mt3 = diag(1, .): y_e = eta~_e,
        Krylov on odd p3 sites.  Otherwise: the whole lattice."""
        if scheme == "SCHUR4D":
            return self.o4, lambda et: self.e4 * self.Amu_inv(self.e4 * et)
        if (scheme == "TEMPORAL_SCHUR" and not self.clover) or scheme == "TEMPORAL_SCHUR3D":
            return self.o3, lambda et: self.e3 * et
        return None, None
