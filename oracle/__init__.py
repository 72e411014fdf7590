"""CPU oracle for the EDFA-preconditioned MHFE-FV solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy restatement of what the paper computes, used to
check the HIP library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the library and its
Python binding never do.  It shares no code with the HIP path: only the
seeded input generators (``paper_2009_13916_amd.inputs``) feed both.

Modules
  mhfe    -- element matrices (Section 2.2, eq. B_ij, Piola map), system
             assembly by the Appendix A formulas, direct solve.
  edfa    -- EDFA stage 1 (Algorithm 1: static / dynamic patterns,
             restricted SPD solves, pre/post filtration, H = G A F, inner
             preconditioner of A_pipi) and stage 2 (Algorithm 2), the
             preconditioner application (eq. EDFA_prec).
  krylov  -- restarted right-preconditioned GMRES / FGMRES.
  adjoint -- transposed-system gradient of a pressure-mismatch loss.

Parity status of each function is stated in its module header.
"""
