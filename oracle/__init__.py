"""FP64 CPU oracle of the lattice Boltzmann scheme of Chatterjee, Strassle, Hosseini and
Karlin, "Consistent lattice Boltzmann model with body force and heat source for
compressible flows of generic fluids".

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP path.

It is a plain, slow, literal transcription of the paper's definitions in float64
NumPy (collide, then stream with np.roll), written for readability:

  lattice      velocity sets, Sec. II C (nearest-neighbour D3Q27 and its 2D restriction)
  equilibrium  Psi functions, product-form f^eq, operator-generated g^eq (Sec. II C)
  bgk          isothermal scheme: Eq. (LBM_f) with f* = f^eq, theta = varsigma^2
  ddf          double-distribution ideal-gas scheme with the Galilean correction Phi
  mlp          learned-collision reference: network, loss, backprop, Adam
"""
