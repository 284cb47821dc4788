"""PEPS norm networks built from seeded inputs with library operations only.

Ket tensors are gathered on the device from dense arrays (ftn_tensor_from_
dense), bra tensors are their Hermitian conjugates (ftn_dagger: Sec. II.D,
Fig. 4a), an optional two-site operator is gathered from its dense array,
and the network is created with the global positions of Fig. 4(a): bras in
reverse site order, then the operator, then the kets.
"""

import torch

from . import ftn
from .ftn import Tensor, Network, dagger

SYM = {"Z2": ftn.Z2, "U1": ftn.U1, "U1xU1": ftn.U1xU1}


def legs_of(site):
    return [([tuple(q) for q in l.charges], list(l.dims), l.dual) for l in site.legs]


def _total(sym, t):
    t = tuple(t)
    return t if len(t) == 2 else (t[0], 0)


def ket_tensors(spec, values, dtype=torch.float64):
    sym = SYM[spec.sym]
    out = []
    for s, site in enumerate(spec.sites):
        dense = torch.as_tensor(values[s], dtype=dtype).to("cuda")
        out.append(Tensor.from_dense(sym, legs_of(site), _total(sym, site.total), dense))
    return out


def operator_tensor(spec, op_dense, dtype=torch.float64):
    """4-leg operator (out_u, out_v, in_v, in_u) from its dense array."""
    sym = SYM[spec.sym]
    phys = spec.sites[0].legs[0]
    ch = [tuple(q) for q in phys.charges]
    dm = list(phys.dims)
    legs = [(ch, dm, 0), (ch, dm, 0), (ch, dm, 1), (ch, dm, 1)]
    dense = torch.as_tensor(op_dense, dtype=dtype).to("cuda")
    return Tensor.from_dense(sym, legs, (0, 0), dense)


def norm_network(spec, kets, op=None, op_sites=None, conv=ftn.LOCAL):
    from synth.workloads import norm_network_bonds, norm_network_positions
    n = spec.n_sites
    bras = [dagger(k) for k in kets]
    tensors = bras + list(kets) + ([op] if op is not None else [])
    bonds = [(t1, l1, t2, l2) for (t1, l1, t2, l2, _) in
             norm_network_bonds(spec, op_sites if op is not None else None)]
    pos = norm_network_positions(n, op is not None)
    return Network(tensors, bonds, conv=conv, positions=pos)
