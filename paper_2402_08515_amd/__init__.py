"""MI355X-native filtered time-domain Krylov eigensolver.

The library (``libkf.so``, C ABI in ``include/kf.h``) computes the eigenpairs
of S v = omega^2 M v (M diagonal) with omega in an interval, using the method
of Nannen & Wess: explicit leapfrog time stepping of M u'' = -S u, filtered
with inverse-Fourier weights, as the operator of a Krylov space; M-orthogonal
Gram-Schmidt and Rayleigh-Ritz on the projected pencil.  ``kf`` is the Python
binding.  Nothing here falls back to the CPU: without the built library every
entry point raises.
"""

__all__ = ["kf"]
