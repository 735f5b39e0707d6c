"""FP64 CPU oracle for phaseless finite-temperature AFQMC on the uniform electron gas.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import or run anything in this package.  It
shares no code with the HIP library: it builds its own plane-wave tables, uses
scipy's Pade-based matrix exponential for the slice propagator, and stabilises
the product with column-pivoted QR (the paper's stratification) at every slice.

Modules
  ueg      -- the system: basis, momentum transfers, kinetic energies, Coulomb
              kernel, one-body remainder of the sum-of-squares form, trial
              chemical potential, Madelung constant (Sec. "Uniform Electron Gas",
              "Computational Details", free-electron trial).
  path     -- one walker's constrained imaginary-time path: force bias, shifted
              propagator, stratified QDT product, stable Green's function and
              log-determinant, phaseless weight (Sec. "Finite-Temperature AFQMC",
              "Numerical Stabilization", "Exploiting the stack structure").
  energy   -- the local energy E_M + E_1 + E_2 with Hartree (Gamma_Q) and
              exchange (Lambda_Q) parts, and the electron number.
  tangent  -- frozen-path derivatives of the weight and the local energy in mu and
              the kinetic scale lambda, by doubled (block-triangular) products
              stabilised like the forward path.

Every function is pinned by a "not gpu" test against something other than
itself (printed values of the paper, closed forms, Fock-space brute force, high
precision products); the one quantity no pin reaches, a full interacting
phaseless path, is "parity unpinned" beyond those invariants.
"""
from . import ueg, path, energy, tangent  # noqa: F401
