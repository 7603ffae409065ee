"""FP64 CPU oracle for the emission-absorption ray march of Ray-trax (arXiv 2511.09389).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the benchmark's CPU-baseline
leg are the only code that may import, call or execute anything in this package. The GPU
product path never routes through it, and it shares no code with the HIP library: no
kernels, headers, helpers, tables or constants. The only thing the two sides both use is
the seeded input generator module, which contains none of the method's arithmetic.

What is computed (paper Sec. 2, Eq. (2) and the paragraphs after it):
  * N_s = ceil(c * dt / ds), optionally capped;
  * N_Omega directions on a Fibonacci (golden-angle) lattice;
  * per ray and substep k: trilinear gather of j at x_k, nearest-neighbour kappa at x_k,
    the update of Eq. (2), index clamping to the box, and a trilinear deposit of the
    post-attenuation I_{k+1} with the same weights, scaled by 4*pi/N_Omega;
  * the multi-source routine is the sum over sources; frequency bins are independent
    copies of the problem (Sec. 2, "Frequency-bin agnosticism").

The surrogate module holds the FP64 reference of the small convolutional network that can
stand in for the march (not part of the paper; the march stays its fallback).

Readings of points the paper leaves open are listed in march.py and in the design notes.
Every function is pinned by tests against closed forms, invariants and brute force.
Parity unpinned: the paper's exact Fibonacci variant, and any field values the paper
shows only in figures (none are printed).
"""

from .march import (  # noqa: F401
    FOUR_PI,
    num_substeps,
    fibonacci_directions,
    trace_single,
    trace_multi,
    trace_bins,
    trace_voxels,
)
from .adjoint import trace_single_vjp, trace_multi_vjp, trace_bins_vjp  # noqa: F401
