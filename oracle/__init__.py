"""Oracle: a plain, slow CPU FP64 implementation of the method.

TEST INFRASTRUCTURE ONLY. This package is imported by ``tests/``, by the
smoke check and by the CPU-baseline leg of the benchmark, never by the
library path. It shares no code with the HIP implementation: tensors are
Python dicts of ``torch.float64`` CPU blocks, every sign is computed by the
definitions written out below, and decompositions call ``torch.linalg``.

Modules and the part of the paper each follows:

* ``symmetry``  Abelian charges and parity (Sec. II.A, II.B)
* ``tensor``    symmetric block-sparse fermionic tensors (Eq. symmetryrule)
* ``ops``       fermionic transposition (Eq. transposition), contraction
                (Eq. standardcontract) under the global and local orderings
                (Secs. II.D, II.E), arrow reversal, fusion (Sec. IV.A)
* ``linalg``    QR / truncated SVD and bond compression (Sec. II.A, II.B)
* ``network``   network contraction along a path, exact and approximate
                (Fig. 1, Secs. II.D, II.E, III)
* ``dense``     brute-force definitions used as pins: Koszul-sign sum over
                all index assignments, swap-gate bosonisation
* ``physics``   Jordan-Wigner Fock space, Hubbard terms (Eq.
                fermi-hubbard-ham), PEPS norm networks (Fig. 4)
* ``amplitude`` amplitudes <n|psi>: projected single-layer networks and the
                sign of fixing the physical legs
* ``adjoint``   reverse-mode derivatives of contractions and networks
"""

from . import symmetry, tensor, ops, linalg, network, dense, physics, amplitude, adjoint

__all__ = ["symmetry", "tensor", "ops", "linalg", "network", "dense", "physics", "amplitude", "adjoint"]
