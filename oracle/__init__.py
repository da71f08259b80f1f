"""Plain FP64 CPU oracle of the mini-batch data-term gradient and weighted prox.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this
package; only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py may import or call it.  It shares no code with the HIP path: the two
meet only in the seeded input generators of the ``synthetic`` package.

Contents (each function cites the passage of arXiv:2307.02043 it follows):

* green      -- truncated Helmholtz Green's kernel, its oversampled
                precomputation on the 2N zero-padded grid, and G / G^H.
* lsmodel    -- BiCGSTAB, the Lippmann-Schwinger forward model H_l, the
                detector residual, the adjoint solve and the mini-batch
                gradient of F_s (Sections 4 and 6), plus the first-Born
                variant and a tangent (J v) solve used only by the pins.
* tvprox     -- discrete TV, its dual, the weighted projection onto the
                nonnegative orthant under tau I + U U^T (Theorem 3.1) and the
                fast dual projected gradient iteration of Section 4.1.
* camera     -- camera sampling of the detector-plane field (an M x M camera
                of its own pitch: trigonometric interpolation of the window's
                field) and its adjoint; a model class that adds it to lsmodel.
* bqnpm      -- the SR1 metric of Algorithm 4.2 and the outer iteration of
                Algorithm 4.1 over the two above.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, a brute-force or dense computation, or an invariant; the paper
prints no worked example for this path, so agreement with its printed
figures is "parity unpinned" (its phantoms and data are not available).
"""
from . import camera, green, lsmodel, tvprox  # noqa: F401
