"""Plain FP64 CPU oracle for spin-restricted CCSDT on full (unpacked) tensors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
It shares no code with the GPU path: its only input is the seeded data from
``cct_inputs``.

Modules
-------
rccsdt    The spin-free (non-orthogonally spin-adapted) RCCSD/RCCSDT working
          equations of the paper's Appendix A (T1-dressed Hamiltonian, RCCSD
          and RCCSDT intermediates, residuals R1/R2/R3 with the paired-index
          permutation operator), the R3 post-processing (symmetrize, purify,
          orthogonalize; Sec. "Removing redundancies"), the Jacobi update with
          orbital-energy denominators, DIIS and the correlation energy.
spinorb   Equation-free brute force in determinant space: FCI, spin-orbital
          projective CC through exp(-T) H exp(T), and the spin-free <->
          spin-orbital amplitude maps (Appendix A spin-free formalism and the
          closed-shell T3 reconstruction formula of the UCCSDT appendix).
blocks    Block- and element-level evaluation of R3 (one output block, or
          sampled output elements, by the term definitions) at sizes where the
          full T3 does not fit in host memory.
counts    Closed-form multiply-add counts of the compact contractions
          (Sec. "Total cost of RCCSDT contractions" and the RCCSDT operation
          count table).
rccsdt_q  The perturbative quadruples correction E_(Q) (Appendix "(Q) energy
          correction"), on full tensors and per occupied or virtual tuple.
rccsdtq   RCCSDTQ on full tensors (Appendix "RCCSDTQ"): the quadruples
          residual, the T4 terms of R2 and R3, the T4 projector.
time_oracle  Wall-clock timing of the oracle on the named workloads (the
          benchmark's CPU baseline figures).
"""
