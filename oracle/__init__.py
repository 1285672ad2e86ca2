"""FP64 CPU oracle for the space-time multilevel quadrature of the monodomain equation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the paper's method computes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP library in
``paper_2105_02007_amd/``; the only common dependency is ``workloads`` (seeded
inputs and workload sizes, no method arithmetic).

Modules and the paper passages they follow:

* ``mesh``       -- uniform Q1 box meshes (Section 3.1, nested meshes h_l ~ 2^-l).
* ``fem``        -- conductivity eq. (AdmV), mass and stiffness matrices and the
                    load vector of the Galerkin semi-discretisation eq. (semi-disc).
* ``tetfem``     -- the same on P1 tetrahedral meshes, with the per-element fibre
                    frame and the point location of the non-nested transfer.
* ``ionic``      -- the cubic ionic current eq. (ionic_term).
* ``stepper``    -- Crank-Nicolson space-time system eq. (st-system) with the
                    reaction term eq. (mono_disc), solved by forward substitution
                    in time with Newton per step; ``allatonce`` solves the whole
                    block system eq. (system_C) + eq. (mono_disc) at once.
* ``kl``         -- discrete Karhunen-Loeve expansion eqs. (algEig), (approxEig),
                    (redEig), (KLlowrank) and the element-midpoint transfer of
                    Section 4.
* ``qmc``        -- randomly shifted rank-1 lattice rules (component-by-component
                    construction) and the normal inverse-CDF map.
* ``estimators`` -- eqs. (SL), (StandardML), (PimpedML) and RMSE estimates.
* ``run``        -- per-sample driver: KL field -> solve -> quantity of interest.

Parity pins live in ``tests/test_oracle_*.py``.  Every function is pinned by
an invariant, closed form, special case or brute-force check there, except the
absolute QoI values of the configured workloads, which are "parity unpinned"
(the paper prints no values; its figures are not part of the text).
"""
