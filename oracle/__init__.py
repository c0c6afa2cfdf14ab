"""Plain, slow, FP64 CPU oracle for particle<->mesh assignment on P1 meshes.

Duque & Espanol, "Assignment of fields from particles to mesh" (arXiv 1610.05258).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product library (the HIP kernels behind the C ABI and its Python binding) never
imports, links or runs it, and this package imports nothing from the product.

Modules
-------
``p1``       the method as the GPU path computes it (particle quadrature for every
             integral, Sec. 2 of the paper read with its own particle quadrature):
             locate, stable binning, scatter of b / w / M^p, FLIP and PIC (Sec. 2.3),
             mass assignment (Sec. 2.4), mesh->particle interpolation (Sec. 2.2) and
             the 1D delta assignment (Sec. 2.2).
``paper1d``  the paper-exact 1D methods of Table 1 (particle hats on the sorted
             particles, consistent mass matrices, exact overlaps and the
             Appendix-B quadrature) and the Sec. 3.1 top-hat experiment.
``metrics``  the error measures E1, E2, L2 of Sec. 3.1 and the volume-weighted L2
             of Sec. 3.3.
``mlp``      FP64 forward/backward of the per-cell warm-start network (not in the
             paper; parity target for the GPU training kernels).
``ns``       the particle fluid solver of Sec. 3.3 (Taylor-Green vortex sheet): P1
             stiffness and gradient operators, a fractional step on the mesh, and the
             P2M / M2P / mid-point advection loop around it.

Every function cites the passage of the paper it follows.  Readings where the paper
is silent or garbled are stated where they are used.
"""
