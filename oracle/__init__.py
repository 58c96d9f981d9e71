"""FP64 CPU oracle for the per-sample evaluation of a fixed-spin single-layer PEPS.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package.  It
shares no code with the HIP library and never imports it.

Modules:
  peps        boundary-MPS contraction (zip-up SVD truncation to Dc), row
              sandwiches, two-row strips, amplitude, gradient blocks, local
              energy (paper Sec. II, Eqs. (1)-(5), Eq. (7))
  brute       exact full contractions on tiny lattices (the plain definition of
              W(S), Eq. (1)) and brute-force local energies
  hamiltonian J1-J2 bond lists and the local-energy assembly E(S) (Sec. II, Eq. (7))
  ed          exact diagonalisation of the open-boundary J1-J2 model (Table I)
  correlations  exchange ratios W(S^{pq})/W(S) for window pairs at any
              distance and the transverse part of <S_p . S_q> (Sec. IV)
  conditioning  per-sample sensitivity of psi, E(S), Delta and the exchange
              ratios to rounding errors in the intermediates (statistical
              condition estimation), which sets the parity bound of samples
              the fixed bounds cannot hold
  metropolis  W^2 Metropolis chains (the stored workload configurations, written
              by make_chains) and one step with shared-environment ratios (Sec. II)
  sweep       one sweep over every nearest-neighbour bond with environments reused
  go          the Eq. (3) sums per spin slice and the Eq. (6) sign update (Sec. III)
  su          simple-update imaginary-time evolution and the D-ramp (Sec. III)
  observables equal-spin counts, <S^z S^z> and structure factors (Sec. IV)

Parity status per function is stated in each module header.
"""
