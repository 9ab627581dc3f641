"""Plain FP64 CPU oracle for the temporally preconditioned Wilson / SW fermion matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or execute anything in this package; only the
test-suite, the smoke check and the benchmark's CPU-baseline leg use it.

It follows Joo, Edwards and Peardon, "An anisotropic preconditioning for the
Wilson fermion matrix on the lattice" (arXiv:0910.0992), written for clarity, not
speed:

* NumPy complex128 on canonical full-lattice arrays (see ``synth``), periodic in
  space, time boundary phase ``b`` (+1 periodic, -1 antiperiodic);
* full 4x4 spin projectors, never half-spinor shortcuts;
* the Sherman-Morrison-Woodbury inverse of the temporal matrix T by literal back
  (forward) substitution as in Sec. II.A, never the axial-gauge rotation;
* even/odd blocks by multiplying with parity masks on the full lattice, never by
  compacting sites.

Direction index convention: 0=x, 1=y, 2=z, 3=t.  The paper's direction 0 (time)
is index 3 here.  Spin matrices are in the Dirac-Pauli basis (gamma_t diagonal,
Appendix C), so P+ keeps the upper two spin components.

Modules:
    dirac     gamma matrices, projectors, sigma_{mu nu}
    wilson    hopping terms D_mu, clover term A, the fermion matrix M (Sec. II)
    temporal  T, T^dagger, their SMW inverses, C_L and C_R (Sec. II.A)
    schemes   parity masks and the four preconditioning schemes (Sec. II.B)
    krylov    CGNR, BiCGStab and the Lanczos condition-number estimate
    force     gradient of |M^-1 eta|^2 w.r.t. the links and the source
    sampled   M at chosen sites and T^-1 on chosen time lines of a large lattice, from
              the functions above called on a small window or a single line

Parity status: every function is pinned by a test in ``tests/test_oracle_*.py``
(free-field momentum space, brute-force dense inverses, gauge covariance,
gamma5-hermiticity, closed-form abelian clover fields, finite differences).
The Lanczos estimate of the smallest singular value is pinned only to 1%.
"""
