"""CPU oracle for the single-layer (nested) CTMRG method of arXiv:2512.14414.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain float64 reference
that the GPU library is checked against.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library itself
never does, and shares no code with it.

Contents
--------
network   nested single-layer network: K, B, X, Y tensors (Eq. XY, Fig. NTN),
          the 4x4 nested cell of a 2x2 PEPS cell (Sec. II C) and its rotations.
ctmrg     multi-site CTMRG on the nested cell: environment start, projectors
          from the bond density matrix (Eqs. PQ, QRSVD), the left-move update
          (Fig. CTMRG b), the sweep of four moves and the spectra test.
double_layer
          the double-layer network of reduced tensors (Eq. Tred) under the
          same CTMRG iteration, and its 2x2 density matrix: the reference
          the nested method converges to as chi grows.
rdm       2x2 reduced density matrix with opened Y tensors (impurities, Sec.
          II B) and the energy E = <H>/<Psi|Psi> (Eq. ExpH).
exact     brute-force references on tiny tori: the state vector, the
          double-layer network of Eq. Tred and the nested network.
adjoint   reverse-mode derivative of E_N(A) (Eq. AD) with textbook QR and
          truncated-SVD adjoints.
mlp       the energy surrogate network (dense, GELU, Adam) in numpy.
lbfgs     L-BFGS with a strong-Wolfe line search and surrogate screening.

Everything runs in float64 on the CPU (torch CPU tensors; numpy for mlp).
"""
