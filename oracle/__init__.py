"""Slow, plain FP64 CPU oracle for the ConvFEM space-angle multigrid transport method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package: only the
test-suite, the smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code with the HIP library (``paper_2301_09991_amd``) and never imports it.

Every function cites the passage of arXiv 2301.09991 (Phillips, Heaney, Chen, Buchan, Pain,
"Solving the Discretised Boltzmann Transport Equations using Neural Networks") that it follows,
by section / equation / appendix.  Where the paper is silent or garbled, the reading adopted is
stated in the docstring of the function that adopts it.

Modules
-------
quadrature  octahedral patch quadrature (section "Discrete Ordinates")
convfem     ConvFEM 1D/2D filters from the averaged finite-element rows (section "ConvFEM",
            Appendix A) and the upwind filters (section "Neural network filters")
transport   halo rule, moments, scatter source, upwind / Petrov-Galerkin residuals
            (eqs. discretised_hfm, Petrov, kxx, kyy, ano-k)
multigrid   space-angle hierarchy, restriction, UpSamp, Jacobi smoothers, sawtooth cycle
            (section "Space-Angle Multigrid", eq. matrix_full)
direct      independent solvers: dense LU, exact upwind sweeps, preconditioned GMRES, Picard
cnn         FP64 reference forward/backward of the small CNN coarse-grid correction
"""
