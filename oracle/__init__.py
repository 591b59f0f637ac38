"""FP64 CPU oracle for the layered-medium Nystrom boundary integral method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

What it computes (Xia, Yuan, Wang, Cai, "Fast boundary integral method for
acoustic wave scattering in two-dimensional layered media"):

* ``medium``     -- Fresnel coefficients, generalized reflection/transmission
                    recursions and the reaction densities sigma (Sec. 3.1,
                    eqs. Rellrecursionup/Rellrecursiondown/generaltransmission,
                    densityinsourcelayer/disity1/disity2).
* ``quadrature`` -- the oracle's own contour quadrature for Sommerfeld
                    integrals (the paper is silent on how they are evaluated).
* ``green``      -- layered Green's function G = delta G^f + sum of the 4L^2
                    non-zero reaction components (eqs. layeredGreensfun,
                    freegreensfun, fourreactions, reflections).
* ``incident``   -- plane wave, background field u^b and boundary data g
                    (Sec. 2, eqs. incidentwave, homogeneousscattering).
* ``nystrom``    -- elements, singular self term I^s, dense matrix K and
                    matvec (Sec. 3.3, eqs. linearSystem, ApproximateComputation,
                    matrixelmemts, Llayerscomponent).
* ``solve``      -- GMRES (unrestarted, x0 = 0) and LU (Sec. 3.3, Sec. 5).
* ``farfield``   -- scattered field by the single-layer representation
                    (eq. integralrep) and top/bottom far-field patterns.
* ``precond``    -- the overlapping domain-decomposition preconditioner
                    (Sec. 4.2), built densely.
* ``kress``      -- beyond the paper's lowest-order rule: a spectrally
                    accurate Nystrom rule (logarithmic product quadrature)
                    for smooth closed scatterers inside one layer.

Readings of garbled or silent passages are marked "reading" in the
docstrings of the modules that depend on them.
"""

from .medium import Medium, nonzero_components  # noqa: F401
