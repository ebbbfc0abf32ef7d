"""FP64 CPU oracle for the azimuthally anisotropic hyperbolic Radon transform (AAHRT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library: the only common module is
``workloads`` (seeded synthetic inputs, none of the method's arithmetic).

Parts
-----
* ``geometry`` -- the discrete axes of the method: stretched axis t' = t^2
  (Section 3.1), the stretch/unstretch interpolators S and S^-1 (Section 3.4,
  read as linear interpolation), the curvature grid, the azimuth of every
  trace and its linear weights onto the uniform theta grid (Section 3.4, the
  theta part of the A1..A4 coefficients), and the FFT length rule.
* ``gfst`` -- oracle-1: Algorithm 1 (Section 3.1), the operator
  R^-1 = S^-1 F1^-1 P F2 S of Section 4, with its step 3 evaluated exactly
  as a direct nonuniform DFT over q (the GFST relation k_q = f'(x^2+y^2),
  theta = arctan(y/x)), and the exact transpose of that pipeline.  This is
  the parity reference for the HIP operators and solver.
* ``timedomain`` -- oracle-2: the conventional Riemann-sum operator of
  Section 5 with linear interpolation in time and azimuth (the operator of
  the equation defining the general AAHRT in Section 2.2, discretised
  directly), and its exact transpose.
* ``fista`` -- oracle-3: forward-backward splitting of Section 4 (soft
  shrinkage), with FISTA momentum, the step from a power iteration, and the
  lambda rule lambda = 0.05 max|L^T d|.
* ``velocity`` -- the automatic anisotropic velocity estimate of Section 3
  (curvature-weighted mean of the Radon cube per intercept and azimuth).
* ``deconv`` -- the deconvolutive AAHRT of Section 4: L_w = W L with W the
  convolution of every trace with the wavelet, and its transpose.
* ``alg2`` -- Algorithm 2 of Section 3.2, the paper's fast velocity stack on a
  regular offset grid, with the (x, y) bilinear interpolation of Section 3.4.
  Not the transpose of L; pinned step by step and by the focusing of events at
  their azimuth-dependent curvature.

Pins: every function here is pinned by ``tests/test_oracle_pins.py`` against
closed forms, invariants, brute force and special cases.  The difference
between oracle-1 and oracle-2 (two discretisations of one continuous
operator) is reported only: parity unpinned for that comparison, as the paper
shows it only as a figure.
"""
from .geometry import Geometry, nfft_rule, theta_weights, stretch_matrix, unstretch_matrix
from . import gfst, timedomain, fista, velocity, deconv, alg2

__all__ = ['Geometry', 'nfft_rule', 'theta_weights', 'stretch_matrix', 'unstretch_matrix',
           'gfst', 'timedomain', 'fista', 'velocity', 'deconv', 'alg2']
