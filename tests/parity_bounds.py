"""Parity tolerances shared by the GPU tests: FP32 kernels against the FP64
oracle on [0, 1] images.

TOL   per-step and operator bound, max-abs, outside near ties: 1e-5.
TAU   width of the near-tie set, in x12 units (S = 12 H_d).  The selection of
      eq. (act) is discontinuous where two candidates of different value have
      (nearly) equal magnitude, so a GPU selection counts as correct where the
      oracle's magnitude of the chosen candidate is within TAU of the oracle's
      minimum.  TAU is 8x the largest |S_gpu - S_oracle| measured at pixels
      whose selection is not in doubt: 1.55e-6 over the 50 states of the
      256 x 256 parity trajectory, 1.85e-6 on uniform random 300 x 517
      images, so TAU = 8 x 1.85e-6 = 1.5e-5 (rounded up).  If every candidate
      is within eps of the oracle's, the GPU's choice is within 2 eps of the
      minimum, so 8x leaves a factor 4.  test_gpu_tau.py measures eps again
      on every GPU run and fails if 8 eps exceeds TAU.
TAU3  the same for the 3-D operator, in x56 units: 8.17e-6 measured at
      settled voxels (runner-up magnitude at least 1e-3 above the minimum) on
      random volumes of 12 x 20 x 70, 9 x 65 x 130 and 30^3, so
      TAU3 = 8 x 8.17e-6 = 6.5e-5, rounded up to 7e-5.
"""
TOL = 1e-5
TAU = 1.5e-5
TAU3 = 7e-5
