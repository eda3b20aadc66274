"""FP64 CPU oracle for the Dynamic DH-MBIR EM step (arXiv 2305.03284).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU path never does.  Shares no code with
the GPU path.

Parity status of each function (what pins it):
  F / FH, back_project ........ Parseval, inverse, delta, explicit DFT sum,
                                adjoint identity against the simulator's A
  normalize ................... mean 0, norm sqrt(p), affine invariance
  remove_tiptilt .............. plane -> 0, residual orthogonal, idempotent
  r_init ...................... hand-computed pixel values of Eq. (3)
  e_step ...................... dense posterior (64x64 inverse) at N=8, a=1
  qggmrf_rho / qggmrf_weight .. finite differences; majorisation on a grid
  solve_pixel_r ............... brute-force grid minimiser; no-prior limit r=s
  r_m_step / phi_m_step ....... pixel-by-pixel sequential ICD at N=8;
                                surrogate decrease; beta=0 limit phi=theta;
                                noise-free frame, w -> 1: the true phase is
                                a fixed point and theta equals it (sign and
                                conjugate conventions of A_phi, A_phi^H, theta)
  em / ddh_frame .............. cost_U non-increasing over 200 iterations;
                                piston invariance; integer-tilt = image shift
  dh_mbir ..................... EM from r = 0 stays at the floor (the loop
                                needs its reset); a lambda = 1 reset makes the
                                result independent of r0; U non-increasing
                                between resets
  grad.reference_gradient ..... loss equals ddh's to 1e-12; FP64 central
                                differences of ddh's loss (sigma_w, sigma_r,
                                beta, a direction in phi0)
  cost_U ...................... dense Gaussian likelihood at N=8, a=1
  strehl ...................... S=1 for constant / tilt residual, Marechal
  phase_rms_diff, rel_l2 ...... hand-computed values on tiny grids; piston and
                                off-pupil invariance; which argument normalises
  noise-free recovery ......... full aperture, dark surround, known r: the
                                true phase is a fixed point of the phase step
                                and pulls a perturbed start back (error
                                reduction); joint EM from a perturbed start
                                does not recover (expected failure, recorded);
                                the circular pupil moves the fixed point
"""
from . import ddh, metrics  # noqa: F401
from .ddh import Params  # noqa: F401
