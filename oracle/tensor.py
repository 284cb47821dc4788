"""Symmetric block-sparse fermionic tensors (Sec. II.A, Eq. symmetryrule).

A leg is an ordered list of sectors (charge, dim) with strictly ascending
charges and a dual flag (0 = '+' outgoing, 1 = '-' incoming). A tensor is an
ordered tuple of legs (the order is part of the tensor, Sec. II.B), a total
charge s(T) and a dict of blocks keyed by tuples of sector indices. A block
is allowed iff sum_i sigma(dual_i) * q_i == s(T); a missing allowed block is
zero. The dense index space of a leg is its sectors concatenated in order.
Blocks are ``torch.float64`` CPU tensors (so autograd can differentiate
through the oracle).
"""

import itertools
from dataclasses import dataclass
from typing import Tuple

import numpy as np
import torch

from . import symmetry as S


@dataclass(frozen=True)
class Leg:
    charges: Tuple[Tuple[int, ...], ...]
    dims: Tuple[int, ...]
    dual: int

    @property
    def nsect(self):
        return len(self.charges)

    @property
    def size(self):
        return int(sum(self.dims))

    def offset(self, i):
        return int(sum(self.dims[:i]))

    def index_of(self, q):
        try:
            return self.charges.index(tuple(q))
        except ValueError:
            return None

    def dim_of(self, q):
        i = self.index_of(q)
        return 0 if i is None else self.dims[i]


def make_leg(sym, charges, dims, dual):
    """Build a leg; sectors are sorted by charge, zero-dim sectors dropped."""
    items = sorted((S.canon(sym, q), int(d)) for q, d in zip(charges, dims) if int(d) > 0)
    for a, b in zip(items, items[1:]):
        if a[0] == b[0]:
            raise ValueError("duplicate charge on a leg")
    return Leg(tuple(q for q, _ in items), tuple(d for _, d in items), int(dual))


def allowed(sym, legs, total, key):
    acc = S.zero(sym)
    for leg, k in zip(legs, key):
        acc = S.add(sym, acc, S.signed(sym, leg.dual, leg.charges[k]))
    return acc == S.canon(sym, total)


def enumerate_keys(sym, legs, total):
    """All allowed sector-index keys, lexicographic order (Eq. symmetryrule)."""
    out = []
    for key in itertools.product(*[range(l.nsect) for l in legs]):
        if allowed(sym, legs, total, key):
            out.append(tuple(key))
    return out


class FTensor:
    def __init__(self, sym, legs, total, blocks=None):
        self.sym = sym
        self.legs = tuple(legs)
        self.total = S.canon(sym, total)
        self.blocks = {} if blocks is None else dict(blocks)

    # --- structure --------------------------------------------------------
    @property
    def ndim(self):
        return len(self.legs)

    @property
    def parity(self):
        return S.parity(self.sym, self.total)

    def keys(self):
        return enumerate_keys(self.sym, self.legs, self.total)

    def shape_of(self, key):
        return tuple(l.dims[k] for l, k in zip(self.legs, key))

    def key_parities(self, key):
        return [S.parity(self.sym, l.charges[k]) for l, k in zip(self.legs, key)]

    def key_charges(self, key):
        return [l.charges[k] for l, k in zip(self.legs, key)]

    def block(self, key):
        b = self.blocks.get(key)
        if b is None:
            b = torch.zeros(self.shape_of(key), dtype=torch.float64)
        return b

    def nnz(self):
        return int(sum(int(np.prod(self.shape_of(k))) for k in self.keys()))

    # --- conversions ------------------------------------------------------
    @classmethod
    def zeros(cls, sym, legs, total):
        t = cls(sym, legs, total)
        for k in t.keys():
            t.blocks[k] = torch.zeros(t.shape_of(k), dtype=torch.float64)
        return t

    @classmethod
    def from_dense(cls, sym, legs, total, arr):
        """Keep the allowed entries of a dense array (leg = sectors concatenated)."""
        arr = np.asarray(arr, dtype=np.float64)
        t = cls(sym, legs, total)
        if arr.shape != tuple(l.size for l in t.legs):
            raise ValueError("dense shape mismatch")
        for k in t.keys():
            sl = tuple(slice(l.offset(i), l.offset(i) + l.dims[i]) for l, i in zip(t.legs, k))
            t.blocks[k] = torch.from_numpy(np.array(arr[sl], dtype=np.float64))
        return t

    def to_dense(self):
        arr = np.zeros(tuple(l.size for l in self.legs), dtype=np.float64)
        for k in self.keys():
            sl = tuple(slice(l.offset(i), l.offset(i) + l.dims[i]) for l, i in zip(self.legs, k))
            arr[sl] = self.block(k).detach().numpy()
        return arr

    def copy(self):
        return FTensor(self.sym, self.legs, self.total,
                       {k: v.clone() for k, v in self.blocks.items()})

    def scaled(self, s):
        return FTensor(self.sym, self.legs, self.total,
                       {k: v * s for k, v in self.blocks.items()})

    def max_abs(self):
        m = 0.0
        for v in self.blocks.values():
            if v.numel():
                m = max(m, float(v.detach().abs().max()))
        return m

    def norm2(self):
        return float(sum(float((v.detach() ** 2).sum()) for v in self.blocks.values()))

    def __repr__(self):
        return "FTensor(%s, ndim=%d, total=%s, nblocks=%d)" % (
            self.sym, self.ndim, self.total, len(self.keys()))
