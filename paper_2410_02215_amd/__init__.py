"""MI355X-native fermionic tensor network contraction (HIP, gfx950).

The library libftn.so (sources in csrc/, C ABI in include/ftn.h) implements
the pairwise fermionic operations of Gao et al., "Fermionic tensor network
contraction for arbitrary geometries": symmetric block-sparse tensors,
fermionic transposition and contraction under the global and local ordering
conventions, fusion, bond compression and network contraction. ``ftn`` is the
ctypes binding; ``autograd`` makes contractions differentiable with torch
through the library's adjoint contraction.
"""

from . import ftn
from .ftn import (Tensor, Network, ftranspose, flip_dual, dagger, fuse, fuse_backward, ftensordot, ftensordot_noalloc,
                  ftensordot_backward, compress_bond, compress_bond_backward, amplitudes, load_library, FtnError,
                  Z2, U1, U1xU1, F64, F32, LOCAL, GLOBAL,
                  GEMM_F64, GEMM_F32, GEMM_BF16X3)

__all__ = ["ftn", "Tensor", "Network", "ftranspose", "flip_dual", "dagger", "fuse", "fuse_backward",
           "ftensordot", "ftensordot_noalloc", "ftensordot_backward", "compress_bond", "compress_bond_backward", "amplitudes", "load_library", "FtnError",
           "Z2", "U1", "U1xU1", "F64", "F32", "LOCAL", "GLOBAL",
           "GEMM_F64", "GEMM_F32", "GEMM_BF16X3"]
