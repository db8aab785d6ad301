"""Float64 CPU oracle of the MADLens hot path (arXiv 2012.07266).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the particle-mesh step and the Born lightcone
projection compute.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It imports nothing from the
HIP library and shares no code, table or constant generator with it.

Modules
  cosmology  background expansion, comoving distance, linear growth,
             kick/drift factors, Eisenstein-Hu no-wiggle linear power
  pm         Zel'dovich initial conditions, CIC paint, Fourier force,
             CIC readout, kick-drift-kick step, full forward run
  lens       Born projection of particle images onto convergence maps
  adjoint    hand-derived vector-Jacobian products of the above
  jvp        hand-derived Jacobian-vector products (forward-mode tangents)

Parity status is stated in each module header.
"""
from . import cosmology, pm, lens  # noqa: F401
