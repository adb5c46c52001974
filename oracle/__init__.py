"""Plain, slow FP64 CPU reference for the P3M periodic-gravity force.

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports, calls or
links this package: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark use it. It shares no code,
tables or constants with the GPU library; it is written from the method's
mathematics (CONCEPT User's Guide, arXiv:1510.07621, Ch. 5 "Parameters" for
the PP/PM/P3M split, cutoff and softening; Ch. 6 for the particle data
layout; Ch. 8 for the drift and kick test designs) and, where the guide is
silent, from the stated readings listed in each module's docstring.

Modules
-------
split      the Gaussian long/short split factor f(r)
pp         O-PP: truncated short-range pair sum (brute force or k-d tree)
pm         O-PM: CIC deposit, FFT Poisson solve with the Gaussian split
           kernel, 4-point finite-difference gradient, CIC interpolation
p3m        O-P3M = O-PP + O-PM (the parity oracle for the GPU force)
ewald      O-EW: direct periodic summation by the Ewald method (the truth)
integrate  kick and drift updates
metrics    per-particle relative force-error statistics
cosmology  background expansion and the comoving kick/drift coefficients
powerspec  power spectrum of the particle density on the PM grid, sigma(R)
adjoint    VJP of the force (pair Hessian-vector sum; mesh adjoint) and of
           the kick-drift-kick leapfrog

Array conventions: positions, momenta, accelerations and forces are float64
arrays of shape (3, N) (structure of arrays, as in the guide's snapshot
layout); masses are a float64 array of shape (N,) or a scalar.
"""
from . import split, pp, pm, p3m, ewald, integrate, metrics, cosmology, adjoint, powerspec  # noqa: F401
