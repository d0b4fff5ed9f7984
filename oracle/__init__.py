"""FP64 CPU oracle for the implicit ohmic-dissipation scheme (Matsumoto, PASJ 2011).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything in this
package.  The HIP library never does, and this package never imports the HIP
library: the two share no code.  Inputs come from ``ohm_inputs`` (seeded
random fields, no method arithmetic).

Modules
-------
ref      -- plain cell-by-cell C primitives (ohm_ref.c) wrapped for numpy:
            face fluxes (eqs. 4-6, 9-11), divergence (8), operator L (13),
            source S (14), residual (20), smoother (19, 21-23), restriction
            and prolongation (section 2.2).
mg       -- the solvers: direct sparse solve, multigrid V-cycle, the paper's
            iterative use of multigrid (eqs. 16-18), V-cycle-preconditioned
            BiCGStab, one Crank-Nicolson step.
amr      -- the composite operator on an AMR hierarchy: coarse-fine ghost
            interpolation and refluxing.
explicit -- the explicit predictor-corrector comparison scheme of section 3.3
            on one level and on an AMR hierarchy.
closed   -- closed forms used as pins: the Fourier symbol of the discrete
            operator, the exact discrete CN and explicit amplification per
            Fourier mode, the continuum decay exp(-eta k^2 t).

Parity status: every function is pinned by a test in tests/test_oracle_*.py,
except the coarse-fine ghost interpolation rule itself (trilinear), which the
paper does not specify: that choice is "parity unpinned" against the paper and
pinned by invariants (linear fields, conservation, uniform refinement) and by
the second-order convergence in the cell width that the paper reports on its
half-refined sinusoid test (Fig. 5).
"""
