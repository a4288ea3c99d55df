"""FP64 CPU oracle for the weighted adjoint NFFT and the forward NFFT.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call this
package: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code with the HIP library; the only module both
sides use is the seeded input generator, which holds none of the method's
arithmetic.

Levels (Kircheis & Potts, arXiv 2302.00414):

* ``ndft``    -- O1, the definition: the sums (2.5)/(2.6), i.e. f = A fhat and
                 h = A^* f with A from (2.7), and the weighted adjoint
                 h^w = A^* W f of (3.6)/(3.7) before any approximation.
* ``nfft``    -- O2, the approximation the method actually evaluates:
                 Algorithm 2.1 (NFFT, A ~ B F D) and Algorithm 2.4 (adjoint
                 NFFT, A^* ~ D^* F^* B^*), written step by step with the
                 Kaiser-Bessel window of ``window``.
* ``weights`` -- O3, Algorithm 3.6: density-compensation factors from the
                 augmented system (3.14) on I_2M, via the normal equations
                 (3.15) (underdetermined) or (3.16) (overdetermined).
* ``bopt``    -- O4, the optimized sparse matrix B_opt of Algorithm 4.3
                 (column-wise least squares with (4.13)/(4.14)) and the
                 reconstruction D^* F^* B_opt^* f of Algorithm 4.4.
* ``window``  -- the Kaiser-Bessel window pair (phi, phi_hat) used by O2.
* ``metrics`` -- the relative errors (5.6).

Everything is float64 / complex128. Every function is pinned by CPU tests
against closed forms, invariants, hand-derived values or brute force.
"""
from . import window, ndft, nfft, weights, bopt, metrics  # noqa: F401
