"""FP64 CPU oracle for periodic voxel homogenization of charge-parametrized shells.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
helpers with the HIP implementation in ``paper_2511_04025_amd``.

The oracle follows the paper (Huang, Liu, Wang, "Shellular Metamaterial Design
via Compact Electric Potential Parametrization", arXiv 2511.04025) in plain
NumPy/SciPy double precision:

* ``field``      -- the truncated periodic charge field, Eq. (6), and its gradient;
                    the distance and occupancy of Eq. (7) (Sec. 4.1);
                    the thickness-from-volume rule (Sec. 4.3, volume constraint).
* ``fem``        -- the 8-node hex element stiffness of a fully solid voxel
                    (Eq. (7), K_0), periodic assembly of K = sum_e K_e, the
                    unit-strain test displacements and right-hand sides (Eq. (8)).
* ``solve``      -- Jacobi-preconditioned CG on the six load cases, and a sparse
                    direct cross-check.
* ``homogenize`` -- the energy form of C^H (Eq. (8)) and the whole forward path.
* ``adjoint``    -- the self-adjoint sensitivities of Eq. (9).
* ``selective``  -- the culled cell problems of Sec. 4.2: active voxels
                    beta > 1e-3, unknowns on the active nodes only, no floor.
* ``multigrid``  -- the coarse grids of Sec. 4.2's hierarchy: periodic
                    trilinear prolongation and Galerkin coarse operators.
* ``metrics``    -- the material metrics and bounds of Sec. 5.2 and the
                    bulk-modulus / Poisson-ratio objective.

Every function is pinned by a ``-m "not gpu"`` test against closed forms,
identities or brute force (see ``tests/test_oracle_*.py``).
"""
