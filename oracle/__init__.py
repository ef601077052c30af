"""Plain FP64 CPU oracle for the matrix-free FEEC operator and its solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; both sides receive the same seeded inputs from ``synth``.

What it computes (paper: "Generalized Yee methods", section 2):
  * the discrete de Rham complex of the paper's eq. (discreteDeRham): integer
    incidence matrices G, C, D with CG = 0 and DC = 0;
  * the mass matrices (M_p)_ij = int (Lambda_i, Lambda_j)_p dx of section 2,
    assembled globally by naive per-element Gauss quadrature (no sum
    factorisation, no fusion);
  * the block operators built from them (mixed Poisson, Hodge Laplacian on
    1-forms, the curl-of-curl P2 = C^T M2 C of section 3) and direct / MINRES
    solves with SciPy.

The spaces are the tensor-product family Q_r^- Lambda^k on a structured
quadrilateral / hexahedral lattice; r = 1 is the paper's generalized Whitney
family of section 4.1.  Degrees of freedom are integrals over lattice cells
(the de Rham map), so incidence is exactly +-1; the paper's average-value
normalisation is a diagonal rescaling exposed by :func:`lattice.cell_measures`.

Parity status per function is listed in each module header.  All functions
are pinned by tests in ``tests/test_oracle_*.py`` against closed forms,
invariants and values printed in the paper.
"""
