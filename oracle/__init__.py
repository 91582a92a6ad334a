"""FP64 CPU oracle for Polarized SARA (Birdi, Repetti & Wiaux, MNRAS 2018).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything under ``oracle/``; the
product path (the HIP library and its Python binding) never does, and the two
share no code.  Every function here is a plain, slow, obviously correct
restatement of the paper's definitions in float64 / complex128 NumPy, each
citing the passage it follows:

* ``kb``      Kaiser-Bessel interpolation kernel and its exact Fourier transform
              (the compact-support kernels of the measurement operator, Sec. 4.1
              eq. meas_op, after Fessler & Sutton 2003).
* ``nufft``   Phi = G F Z per Stokes column, the Stokes-to-brightness mixing L
              (Sec. 2.1, eq. after RIME) and phi / phi^dagger (eq. meas_op).
* ``sara``    Daubechies filters by spectral factorisation, periodised 2-D DWT,
              and the SARA frame Psi = (1/3)[Dirac, Db1..Db8] (Sec. 3.1).
* ``prox``    the closed-form projections and thresholding of Sec. 3.3.
* ``pd``      Algorithm 1 (primal-dual) and Algorithm 2 (reweighting), the
              power iteration for the step-size condition of Sec. 3.3.3.
* ``metrics`` SNR, NRMSE, polarisation error image / N_p, stopping quantities
              (Sec. 4.3-4.6).

Readings of passages that are ambiguous or garbled are listed in each module
header.  Functions with no independent pin say "parity unpinned".
"""
