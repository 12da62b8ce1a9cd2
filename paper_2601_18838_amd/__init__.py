"""MI355X-native reciprocal-space Kroneckerised PME (SKP-PME).

The hot path -- B-spline spread, the Sum-of-Kronecker-Products reciprocal
operator applied as mode products on the matrix cores, gather of potentials
and forces, energy -- runs in hand-written gfx950 HIP kernels behind the
C ABI declared in ``include/kpme.h``.  ``kpme`` is the thin Python binding.
"""
