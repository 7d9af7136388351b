"""CPU oracle for the PDE-compressed Cartesian-Taylor FMM translation operators.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it; the only module both sides use is the
seeded input generator ``workloads`` (geometry only, none of the method's
arithmetic).

Everything here is plain and slow on purpose: NumPy float64 / complex128, Python
``fractions`` for exact rational PDE matrices, and mpmath (50 digits) for
derivative tables that pin the float64 ones.  Each function cites the passage of
Fernando & Kloeckner, "Automatic Synthesis of Low-Complexity Translation
Operators for the Fast Multipole Method" (arXiv 2305.17867) that it follows.

Modules
  multiindex   multi-index sets M(p), the graded ordering, the kept set J
  kernels      kernels G, their PDE operators, direct sum eq. (1), derivative tables
  compression  PDE-coefficient matrix P, h, j-bar, decompression matrix M (Sec. 3.1)
  taylor       uncompressed Cartesian Taylor P2M / M2L / L2P (Sec. 2)
  compressed   compressed P2M / M2L / L2P, the scaled form (Sec. 4.1.1), the FFT form
               (eq. convolution_m2l)
  adjoint      gradients of the direct sum and transposes of the discrete FMM map

Parity status: every function is pinned by a ``-m "not gpu"`` test against
closed forms, exact symbolic differentiation, theorems of the paper or brute
force; none is "parity unpinned".
"""
