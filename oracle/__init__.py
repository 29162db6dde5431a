"""CPU FP64 oracle for the phaseless-AFQMC walker step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py, never by the GPU library. It shares no code with the
HIP path; both sides take their inputs from paper_2003_01831_amd.synth.

Parity status per function (pins in tests/test_oracle_*.py):
  afqmc.local_energy_plain / local_energy_half / overlap   pinned (FCI brute force)
  afqmc.one_body_corrected                                 pinned (FCI operator identity)
  afqmc.taylor_apply                                       pinned (scipy expm + bound)
  afqmc.run (propagation, weights, QR)                     pinned (HS identity on FCI
                                                           vectors, L=0 closed form,
                                                           invariants, E_shift invariance)
  afqmc.energy_grad / mixed_rdm1                           pinned (central differences,
                                                           explicit 1-RDM from FCI)
  afqmc.comb / eshift_update / caps in run                 pinned (hand example, floor/ceil
                                                           counts, unbiasedness, limits)
  afqmc.back_propagate / back_propagated_rdm1              pinned (many-body matrix element
                                                           in the FCI space, L=0 ground-state
                                                           density, invariances, walk
                                                           bookkeeping incl. comb ancestry)
  msd.overlap / local_energy, run(msd=...)                 pinned (CI-vector matrix elements in
                                                           the FCI space, orthonormality,
                                                           zero variance of a complete
                                                           expansion, one-determinant limit)
  kpoint.* (general complex Cholesky walk, k-point blocks) pinned (determinant-space matrix
                                                           elements, operator identity for h'
                                                           and the two fields, short-time HS
                                                           limit, force-bias cancellation,
                                                           Bloch transform of a supercell)
  philox.philox4x32_10                                     pinned (published KAT vectors)
"""
