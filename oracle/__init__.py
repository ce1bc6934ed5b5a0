"""FP64 CPU oracle for randomized-block-Krylov Tucker (rBKI-TK) and its
hierarchical tensor-ring variant (rBKI-TK-TR), after Qiu, Sun, Zhou and Zhao,
"Towards Efficient and Accurate Approximation: Tensor Decomposition Based on
Randomized Block Krylov Iteration" (arXiv 2211.14828).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may.  It shares no code with the HIP implementation; the two meet
only through the seeded input generators in ``synth`` (which hold none of the
method's arithmetic) and through the published definition of the Philox4x32-10
counter-based generator, which each side implements on its own.

Everything is plain NumPy/SciPy in float64 (the paper's MATLAB runs are in
double), written for a reader to check against the paper by eye: no blocking,
fusion or reordering beyond what the paper's definitions and algorithms state.

Modules
-------
philox   : Philox4x32-10 and the Box-Muller Gaussian sketch matrix Omega.
tensor   : mode-n unfolding, folding and mode-n products (Table 1, eq. (1)).
rbki     : Alg. 1 (rBKI tensor sketching), Alg. 2 (rBKI-TK), and the q=0 /
           power-iteration special cases the paper compares against.
thosvd   : truncated HOSVD, the deterministic benchmark of Sec. 4.
trsvd    : TR-SVD, tensor-ring reconstruction and Alg. 3 (rBKI-TK-TR).
metrics  : Fit, RErr (Sec. 4) and projector distances.

Parity-unpinned items (no value fixed by the paper or by mathematics):
signs and in-cluster order of factor columns, TR cores (gauge freedom; only
reconstructions are compared), the 4th-order power-functional case of Table 4.
"""
