"""The operation counts of App. B, re-derived from their parts: an SU(3) matvec, a spin
reconstruction, a 4-spinor sum, the clover block and the SMW substitution and Woodbury steps
(FLOPs as the paper counts them: a complex multiply 6, a complex add 2, spin projections free).
The totals the paper prints (tests/golden/appB_operation_counts.txt) must follow from those
parts; a garbled term fails here."""
import os

import pytest


def _golden():
    """The printed counts: {name: count} for per-site values, {name: (a, b)} for a N_t + b,
    and the printed ratios {(num, den): (leading, 1/N_t coefficient)}."""
    per_site, per_apply, ratios = {}, {}, {}
    path = os.path.join(os.path.dirname(__file__), "golden", "appB_operation_counts.txt")
    with open(path) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            f = line.split()
            if f[0] == "per_site":
                per_site[f[1]] = int(f[2])
            elif f[0] == "per_apply":
                per_apply[f[1]] = (int(f[2]), int(f[3]))
            elif f[0] == "ratio":
                num, den = f[1].split("/")
                ratios[(num, den)] = (float(f[2]), float(f[3]))
    return per_site, per_apply, ratios


SITE, APPLY, RATIOS = _golden()


CMUL, CADD = 6, 2
MATVEC = 3 * (3 * CMUL + 2 * CADD)          # three rows: 3 complex multiplies, 2 adds
RECONS = 6 * CADD                            # 6 complex adds (2 spin-colour components)
SUMVEC4 = 12 * CADD                          # sum of two 4-spinors: 12 complex components
CLOVER = SITE["clover"]                      # per site, stated by the paper
AXPY = 48                                    # scaling and subtraction of two 4-spinors


def hop(nd, n_gamma_star=2):
    """Projected hopping term in nd dimensions: forward and backward per dimension."""
    return 2 * nd * (n_gamma_star * MATVEC + RECONS) + SUMVEC4 * (2 * nd - 1)


def subst(nt):
    """Back substitution on one spin component: one scaling, then nt - 1 steps of a matvec, a
    subtraction and a scaling."""
    return 6 + (nt - 1) * (MATVEC + 6 + 6)


def woodbury(nt):
    """The rest of SMW per spin component: a matvec and a subtraction per slice."""
    return (MATVEC + 6) * nt


def c_per_line(nt):
    """C_L or C_R per spatial site pair (V_s/2): two spin components, plus reconstruction and
    projector sum on every site of the checkerboard."""
    return 2 * (subst(nt) + woodbury(nt)) + (12 + 48) * nt


def test_parts():
    assert MATVEC == 66
    assert RECONS == 12 and SUMVEC4 == 24


def test_hopping_terms():
    assert hop(4) == SITE["hop_4d"]  # 4D D^oe
    assert hop(3) == SITE["hop_3d"]  # 3D D_s


def test_4d_schur():
    assert (2 * (hop(4) + CLOVER) + AXPY, 0) == APPLY["schur4d_clover"]
    # Wilson, mu - D^oe D^eo / (4 mu): the paper prints 2668, but its own terms (an AXPY and two
    # 4D hops) add up to 2688; the Wilson ratio of App. B is then 3432/2688 = 1.277 at large N_t
    wilson = AXPY + 2 * hop(4)
    assert wilson == 2688
    assert wilson - APPLY["schur4d_wilson"][0] == 20


def test_printed_ratios():
    """Each printed cost ratio follows from the printed counts to the digits it shows."""
    for (num, den), (lead, inv) in RATIOS.items():
        a, b = APPLY[num]
        a2, _ = APPLY[den]
        digits = len(str(lead).split(".")[1])
        assert round(a / a2, digits) == lead, (num, den)
        assert round(-b / a2, 3) == inv, (num, den)


@pytest.mark.parametrize("nt", [1, 16, 64, 128, 256])
def test_preconditioner_and_ilu(nt):
    def printed(name):
        a, b = APPLY[name]
        return a * nt + b
    assert subst(nt) == 78 * nt - 72
    assert woodbury(nt) == 72 * nt
    assert c_per_line(nt) == printed("c_line")
    # clover ILU: 5 vector adds, 8 applications of C, A and D_s twice (per V_s/2)
    ilu = 5 * 24 * nt + 8 * c_per_line(nt) + (2 * CLOVER + 2 * hop(3)) * nt
    assert ilu == printed("ilu_clover")
    # Wilson ILU: one vector add, 4 applications of C, D_s twice
    assert 24 * nt + 4 * c_per_line(nt) + 2 * hop(3) * nt == printed("ilu_wilson")


@pytest.mark.parametrize("nt", [16, 128, 256])
def test_dirac_basis_and_axial_gauge(nt):
    """Dirac basis: no reconstruction or projector sum in C (60 per site, 8 C); axial gauge: no
    matvec in the nt - 1 substitution steps (66 per step and spin component, 8 C)."""
    a, b = APPLY["ilu_clover"]
    ilu = a * nt + b
    saved = 8 * 60 * nt + 8 * 2 * MATVEC * (nt - 1)
    a, b = APPLY["ilu_clover_db"]
    assert ilu - saved == a * nt + b


def test_cutoff_saving():
    """Cutoff at k slices: a matvec and a subtraction per slice and spin component, per C."""
    k = 40
    per_c = 2 * (MATVEC + 6) * k
    assert per_c == 144 * k
    assert 8 * per_c == 1152 * k and 4 * per_c == 576 * k
