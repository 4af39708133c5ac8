"""FP64 CPU oracle for the semilinear lens solve -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the GPU
library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

It follows Rogers & Fiege (2011), "Gravitational Lens Modeling with Genetic
Algorithms and Particle Swarm Optimizers":

* ``lens``      -- thin-lens mapping (Eq. 1), SIE deflection (Eqs. 10-11),
                   SIS (Sec. 4), plus external shear (not in the paper).
* ``operators`` -- bilinear lens operator L and its transpose (Sec. 2.1,
                   Sec. 2.2), PSF blur B and B^T (Sec. 2.2), regularisation H
                   (Eq. 7).
* ``solve``     -- Tikhonov system (Eq. 7, Eq. 13-14 with x0 = 0), dense
                   Cholesky and matrix-free CG, chi^2 (Eq. 4), SVD filter
                   factors (Eqs. 15-19).
* ``lcurve``    -- arclength-parameterised cubic-spline L-curve and maximum
                   curvature (Sec. 2.6, Eq. 20).
* ``mock``      -- analytic sources, Gaussian PSF and noisy mock images
                   (Sec. 2.3).
* ``mlp``       -- FP64 reference of the surrogate MLP (not in the paper).
* ``ga``        -- one generation of the simplified Ferret GA (Sec. 3.1.1,
                   App. A.1) driven by pre-drawn random numbers.
* ``coracle``   -- ctypes wrapper of ``csolve.c``, the same matrix-free FP64
                   solve written in plain C (OpenMP over members), used as the
                   timed CPU baseline.

Every function states the passage it follows.  Where the paper is silent the
module docstrings state the reading taken.
"""
