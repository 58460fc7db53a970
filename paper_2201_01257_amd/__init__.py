"""MI355X (gfx950) block-sparse tensor contraction over tiled, spin-blocked index spaces.

The hot path of TAMM (arXiv 2201.01257): block-sparse tensors over tiled index spaces with
spin-block sparsity, and the contraction ``out(..) = beta*out(..) + alpha * lhs(..) * rhs(..)``,
executed by hand-written HIP kernels (GPU tile-pair screening, index-permuted LDS gathers,
MFMA products, atomic-free epilogue) behind a C ABI (include/tamm_mi.h).  This package is the
thin Python binding; importing it does not load the native library, the first call does, and
fails loudly if the library has not been built.
"""

from .core import (Denominator, Group, Plan, Space, TammError, Tensor, contract, contract_cache_clear,  # noqa: F401
                   contract_cache_count)

__all__ = ["Space", "Tensor", "Plan", "Group", "contract", "contract_cache_count", "contract_cache_clear", "Denominator",
           "TammError"]
