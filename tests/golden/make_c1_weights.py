"""Write tests/golden/c1_weights.npz: density-compensation weights of
Algorithm 3.6 computed by the CPU oracle (oracle/weights.py) for the two
2-D, M = 32 correctness workloads the GPU tests reconstruct with.

  w_c1   N = 4096 uniform random nodes (seed 1): |I_2M| = N, branch (3.15),
         the dense minimum-norm least-squares solve of A_2M^T w = e_0
         (badly conditioned: cond(A_2M) ~ 3e7, the weights reach ~1e7 / N)
  w_c1b  N = 16384 uniform random nodes (seed 7), the size of the random-node
         experiment of Example 5.2 (N_t = 2^(9-d) per dimension): |I_2M| < N,
         branch (3.15) by CG with exact-sum (O1) products, tolerance 1e-13

Run from the repository root:  python tests/golden/make_c1_weights.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import weights as ow  # noqa: E402
from paper_2302_00414_amd import workloads as wl  # noqa: E402

M = 32
x1 = wl.uniform_nodes(4096, 2, 1)
w1 = ow.weights_lstsq(x1, M)
x2 = wl.uniform_nodes(16384, 2, 7)
w2, info = ow.weights_cg(x2, M, "ndft", tol=1e-13)
eps1, eps2 = ow.residual(x1, w1, M), ow.residual(x2, w2, M)
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_weights.npz")
np.savez(out, w_c1=w1, w_c1b=w2, eps_c1=eps1, eps_c1b=eps2)
print(f"wrote {out}: eps c1 {eps1:.3g}, c1b {eps2:.3g} ({info['iterations']} CG iterations)")
