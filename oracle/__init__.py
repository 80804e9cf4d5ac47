"""Plain FP64 CPU oracle of CP-ALS-QR (Minster, Viviano, Liu, Ballard,
"CP Decomposition for Tensors via Alternating Least Squares with QR
Decomposition", arXiv:2112.10855).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It exists only to check the GPU path.
Only the test suite, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
imports, links or calls anything in here, and nothing in here calls the GPU
library: the two share no code, no tables and no helpers.

Everything is written to be read against the paper by eye: float64 numpy,
library primitives (matmul, reduced Householder QR, SVD, triangular and
Cholesky solves) used as single steps, and no blocking, fusion or reordering
beyond what the paper's definitions and algorithms state.

Modules
  tensor     -- Kronecker / Khatri-Rao / Hadamard products, mode-n unfolding,
                TTM, Multi-TTM, Kruskal reconstruction (paper section 2.2, 2.3)
  cp_als_qr  -- Alg. 2 (CP-ALS-QR and CP-ALS-QR-SVD) step by step (section 3.1)
                with both error forms (section 3.3.1)
  cp_als     -- Alg. 1 (CP-ALS and CP-ALS-PINV), the normal-equations
                comparator (section 2.3)
  kruskal    -- Alg. 2 and Alg. 1 on a Kruskal-form input (section 3.3.2) and
                the structured QR of the Khatri-Rao product of triangular
                factors (section 3.3.3, eq. kr-id)
  costs      -- the flop model of section 3.2 (eq. QRcost, eq. TTMcost)
  precision  -- bit-level bfloat16 rounding and split-bfloat16 products, the
                reduced-precision Multi-TTM forms the GPU offers
  learned    -- the learned initializer: tensor sketch, three-layer MLP,
                Kruskal-form loss and its gradient, Adam

Pins.  Every function here is pinned by ``tests/test_oracle_*.py`` to facts
the paper and the mathematics fix (brute-force index loops, identities,
invariants, closed forms), never to itself.  Functions without such a pin say
"parity unpinned" in their docstring.
"""

from . import tensor, cp_als_qr, cp_als, costs, precision, learned, kruskal  # noqa: F401
