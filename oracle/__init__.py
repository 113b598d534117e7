"""CPU oracle for MG-MLMC++ (Frommer & Nasr Khalil, "MG-MLMC++ as a Variance
Reduction Method for Estimating the Trace of a Matrix Inverse").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128
implementation written to check the HIP library against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product path (``paper_2303_11512_amd``) never does, and the two
share no code.

Modules
-------
rng     counter-based SplitMix64 noise (isotropic vectors, Sec. 1 eq. random_props)
dirac   the Schwinger (2D Wilson-Dirac, U(1)) operator as a scipy sparse matrix
mg      aggregation multigrid setup, Galerkin operators, and the reference
        preconditioner (SAP smoother, K-cycle) used only to pin the HIP solver
trace   Alg. 1 (plain Hutchinson), Hutch++ (Sec. 2.4), MG-MLMC (Sec. 3.1) and
        MG-MLMC++ (Alg. 2), run step by step in the paper's order
cnn     the small convolutional initial-guess network (forward, backward, Adam)

Parity status of each function is stated in its docstring; a function whose
result nothing in the paper or the mathematics fixes says "parity unpinned".
"""
