"""CPU oracle for the MLMC Darcy-flow hot path (test infrastructure only).

This package is a plain, slow, single-threaded FP64 restatement of what the
GPU library computes, written from Park & Teckentrup, "Improved Multilevel
Monte Carlo Methods for Finite Volume Discretisations of Darcy Flow in
Randomly Layered Media" (arXiv 1506.04694).  It exists to check the GPU path:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The GPU library never calls it, and it shares no
code with the GPU library (kernels, headers, helpers or tables).

Modules and the passages they follow:

* ``philox``   -- counter-based normals feeding Example 1 / Example 2
                  (the paper names no generator; Philox4x32-10 of Salmon et
                  al., SC'11, is this build's choice, restated from its
                  published definition).
* ``geometry`` -- the random layer partition of Section 2 and the layer
                  shapes of Section 3.4.
* ``field``    -- Example 1 (piecewise constant log-normal), Example 2 with
                  eq. (2.3) sampled by circulant embedding (Section 3.4),
                  the plain coarse sample of eq. (3.6) and the Coarse Grid
                  Variates sub-samples of Section 4.1.
* ``fv``       -- the cell-centred finite volume system eq. (3.3) with
                  harmonic-mean faces (Sections 3.1 and 3.4) and the
                  Model Problem 2 boundary conditions, eq. (3.11).
* ``solve``    -- the exact discrete solution by a sparse direct solve.
* ``qoi``      -- the outflow functional M^(2) of Model Problem 2.
* ``mlmc``     -- the estimators eq. (3.6), eq. (3.7), eq. (4.1), eq. (4.2).

Every function is pinned by ``tests/test_oracle_*.py`` against facts fixed
by the paper or by mathematics (closed forms, invariants, brute force,
library routines), never against itself or the GPU path.
"""
