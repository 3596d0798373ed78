"""Plain FP64 CPU oracle for APLICUR -- TEST INFRASTRUCTURE ONLY.

This package is a slow, obviously-correct NumPy/SciPy restatement of what the
APLICUR hot path computes (Huh, Cartis, Nakatsukasa, "Adaptive LSQR
Preconditioning from One Small Sketch", arXiv 2604.05065).  It exists only to
check the HIP implementation.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2604_05065_amd``) never does, and the two share no code.

Modules
-------
rng      counter-based SplitMix64 stream that draws the sparse sign embedding
         (Definition 5.1) and the Gaussian probe vectors of the randomized
         2-norm bound (Sec. 5.3.1).
lsqr     one LSQR phase on the augmented, right-preconditioned operator
         A_mu P^{-1} (Sec. 2.2 and Sec. 5.3.2), Paige-Saunders recurrences.
cur      LU-with-partial-pivoting pivot selection, augmentCUR (Alg. 7),
         augmentQR (Alg. 9), the CUR preconditioner (Alg. 2) and the rho
         estimator (Sec. 5.3.1).
aplicur  the full adaptive procedure (Alg. 3) plus plain damped LSQR.
dense    closed-form references: dense-QR solution of the augmented problem
         (Sec. 2.1), the normal-equation residual, and the adjoint gradient.

Parity status of each function is stated in its docstring.  The adaptive
schedule itself (rank sequence, phase lengths) has no printed values in the
paper: it is "parity unpinned" against the paper and is pinned only through
the closed forms and invariants tested in ``tests/test_oracle_*.py``.
"""
