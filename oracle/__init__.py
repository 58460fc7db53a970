"""FP64 CPU oracle for block-sparse tensor contraction over tiled, spin-blocked index spaces.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call, link or execute
this package; only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP path: its own tiling, its own block-storage rule, its own
contraction loop.  It is deliberately plain and slow: nested Python loops over tiles, with one
``numpy.einsum`` per surviving tile pair, in float64.

What it follows (arXiv 2201.01257, "TAMM: Tensor Algebra for Many-body Methods"):

* tiled index spaces, fixed or explicit tile lists, tensors as blocks over the Cartesian
  product of tiles (Sec. III-A, Fig. 1);
* spin-blocked storage where structurally zero blocks are not stored, and a user-supplied
  non-zero check used both for allocation and for operation execution (Sec. III-A);
* the contraction operation ``C(..) += alpha * A(..) * B(..)`` of the operation grammar
  (Sec. III-A, Fig. 3, grammar rule 8) and its ``=`` / ``+=`` / ``-=`` forms;
* the CCSD doubles terms, the intermediate factorisation of Eqs. (cc9)-(cc11) and its TAMM
  form (Eq. tamm_cc11), spin-explicit sub-spaces (Eq. tamm_cc-Spin), Sec. IV-A-1;
* the SetOp and AddOp (with a label permutation) of the same grammar (Fig. 3, rules 5-7);
* the orbital-energy-denominator update that turns a doubles residual into new amplitudes
  (the Jacobi step of CD-CCSD, named in Sec. IV-B-1);
* the ladder over integrals rebuilt from Cholesky vectors, Eq. (cc12), with the rebuilt tensor
  as a lambda tensor whose blocks are computed on demand (Sec. III-A).

Readings taken where the paper is silent are listed in the module docstrings they affect.

Pins: every function here is checked by the ``-m "not gpu"`` tests against something other
than itself (dense brute force, a BLAS GEMM special case, the Eq. (cc9)-(cc11) identity,
closed-form block counts, the worked tiling example of Fig. 1, invariants, finite
differences).  The operand splits of the mixed-precision paths (``oracle.split``) are pinned
by their own tests.  The mixed-precision contractions themselves are checked against this
float64 oracle element by element within a worst-case bound derived from the split definitions
and the rounding of the matrix-core instructions, which is measured on the device on inputs
whose exact sums are known (``tests/mixed_bound.py``, ``tests/test_gpu_mfma_rounding.py``).
"""

from .tiling import Space, spin_conserving
from .blocksparse import BlockTensor, LazyBlocks, contract, screen, denominator_update, parse_labels
from .adjoint import contract_vjp
from .elementwise import add, set_value
from .cholesky import cholesky_ladder, v_from_cholesky, spin_diagonal

__all__ = [
    "Space",
    "spin_conserving",
    "BlockTensor",
    "LazyBlocks",
    "contract",
    "screen",
    "denominator_update",
    "parse_labels",
    "contract_vjp",
    "add",
    "set_value",
    "cholesky_ladder",
    "v_from_cholesky",
    "spin_diagonal",
]
