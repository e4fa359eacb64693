"""FP64 CPU oracle for the TILD particle-mesh step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it, and it shares no code with the HIP path: positions, assignment
weights, transforms, k-space factors, forces, bonds, noise and updates are all
computed here independently, in float64, from the paper's definitions.

Passages followed (paper sections and equations):
  * microscopic densities, Eq. rhohat;
  * harmonic bonds, Eq. bonds;
  * non-local Flory repulsion, Eq. fh; Helfand compressibility, Eq. HelfandP;
  * Gaussian smearing and the equivalent local forms with sigma^2 = 2 a^2,
    Eqs. smearRho, fhF, HelfandF;
  * the particle-to-mesh force route (spread -> FFT -> multiply -> inverse
    FFT -> interpolate with the same spline weights), Eq. PMM and Fig. pmm;
  * the Euler-Maruyama update form, Eq. EM and the Integrator list;
  * the structure factor, Eq. sk.
Readings where the paper is silent are listed next to each function.
"""

from .tild_ref import *  # noqa: F401,F403
from .philox_ref import philox4, philox4x32, gaussian_noise  # noqa: F401
