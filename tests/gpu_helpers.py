"""Bridges between oracle tensors and the HIP library for parity tests.

Only the seeded inputs cross over: a structure (legs, total) and a dense
random array. The library builds its tensor from the dense array with its
own block enumeration; results are read back and compared with the oracle.
"""

import numpy as np
import torch

from oracle import symmetry as S
from oracle.tensor import FTensor, Leg

SYM = {S.Z2: 0, S.U1: 1, S.U1U1: 2}


def legs_abi(legs):
    return [([tuple(q) for q in l.charges], list(l.dims), l.dual) for l in legs]


def to_gpu(T, dtype=torch.float64):
    import paper_2410_02215_amd as P
    dense = torch.from_numpy(T.to_dense()).to(device="cuda", dtype=dtype)
    tot = tuple(T.total) + ((0,) if len(T.total) == 1 else ())
    return P.Tensor.from_dense(SYM[T.sym], legs_abi(T.legs), tot, dense)


def gpu_legs(sym, G):
    out = []
    for chs, dims, dual in G.legs():
        qs = [(c[0],) if sym != S.U1U1 else (c[0], c[1]) for c in chs]
        out.append(Leg(tuple(qs), tuple(dims), dual))
    return out


def from_gpu(sym, G):
    """Oracle FTensor with the GPU tensor's structure and values."""
    inf = G.info()
    tot = (inf["total"][0],) if sym != S.U1U1 else tuple(inf["total"])
    legs = gpu_legs(sym, G)
    dense = G.to_dense().double().cpu().numpy()
    return FTensor.from_dense(sym, legs, tot, dense)


def assert_same_structure(T, G):
    """Block keys and offsets bit-exact against the oracle enumeration."""
    keys, offs, shapes = G.blocks()
    ok = T.keys()
    assert keys.shape[0] == len(ok)
    if len(ok) and T.ndim:
        np.testing.assert_array_equal(keys, np.array(ok, dtype=np.int32))
    sizes = [int(np.prod(T.shape_of(k))) for k in ok]
    np.testing.assert_array_equal(offs, np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))


def flat_blocks(T):
    parts = [T.block(k).detach().numpy().ravel() for k in T.keys()]
    return np.concatenate(parts) if parts else np.zeros(0)


def rounded_f32(T):
    """Copy of an oracle tensor with every entry rounded to FP32 and back.

    An FP32 path starts from these values, so comparing it with the oracle
    on them isolates the arithmetic of the path from the input rounding.
    """
    out = FTensor(T.sym, T.legs, T.total)
    for k in T.keys():
        out.blocks[k] = T.block(k).to(torch.float32).to(torch.float64)
    return out
