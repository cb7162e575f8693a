"""Plain FP64 CPU oracle for the L-tsNET gradient (test infrastructure).

This package is the yardstick that the GPU path is checked against. It is not
part of the product: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import or call it, and the GPU path never routes through
it. It shares no code with the HIP library; the only common module is the
input generator package ``synth``, which holds none of the method's arithmetic.

Modules, each citing the passage of the paper it follows:

* ``tiebreak``   -- the counter-based hash that makes "ties broken randomly"
                    reproducible (SplitMix64 finaliser).
* ``neighbours`` -- partial BFS k-nearest-neighbour selection (Sec. 3.1;
                    Algorithm 3, C0 block).
* ``perplexity`` -- conditional probabilities p_{j|i} with the bandwidth set by
                    the perplexity (Eq. 3).
* ``affinities`` -- symmetric joint probabilities p_ij (Eq. 2) in CSR form.
* ``gradient``   -- exact O(n^2) gradient of the cost (Eq. 1, 6, 8), the cost
                    itself and the per-coordinate finite-difference helper.
* ``interp``     -- FP64 FFT-accelerated interpolation of the kernel sums
                    (Sec. 2.3, Sec. 3.3), the approximation the GPU path uses.
* ``step``       -- the vertex move (Algorithm 3, last step of the loop).
* ``pmds``       -- the Pivot MDS starting layout (Algorithms 1-3, first step).
* ``metrics``    -- neighbourhood preservation (r = 2) and stress of a layout
                    (Sec. 4.3.1, Sec. 4.3.2).
* ``quadtree``   -- Barnes-Hut quadtree sums of the repulsion and entropy terms
                    (BH-tsNET and FIt-tsNET, Algorithms 1-2, Eq. 7).

Parity pins (tests marked ``not gpu``) tie each function to something other
than itself: closed-form BFS distances, brute-force selection, library root
finding, finite differences of the cost, zero-sum and symmetry invariants,
polynomial exactness of the interpolation and library FFT convolution.
"""

from . import tiebreak, neighbours, perplexity, affinities, gradient, interp, step, pmds, metrics, quadtree  # noqa: F401
