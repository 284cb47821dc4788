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


def energy_gradient(spec, kets, terms, paths, chi=0, checkpoint=0):
    """E = sum_t <psi|G_t|psi> / <psi|psi> and dE/d(ket tensors), by the
    library's network backward pass (ftn_contract_network_grad).

    ``terms``: list of (G Tensor, (u, v)); ``paths``: {None: norm path,
    (u, v): path of that term}. Each network is <psi|psi> or <psi|G_t|psi>
    with the bras made by ftn_dagger from the kets; the gradient of a network
    with respect to a ket collects its ket slot and, through the adjoint of
    the Hermitian conjugate (the same relabelling: ftn_dagger), its bra slot.
    With N = <psi|psi> and X_t the terms, dE = sum_t dX_t / N - E dN / N; the
    combination is a sequence of ftn_tensor_axpy calls with scalar weights.
    Returns (E, [gradient Tensor per ket]).
    """
    n = spec.n_sites

    def value_and_ket_grads(op, sites):
        net = norm_network(spec, kets, op=op, op_sites=sites)
        m, e, g = net.contract_grad(paths[tuple(sites) if sites is not None else None], chi=chi,
                                    checkpoint=checkpoint)
        # slots: bra s -> s, ket s -> n + s
        return m, e, [ftn.axpy(1.0, dagger(g[s]), g[n + s]) for s in range(n)]

    mN, eN, gN = value_and_ket_grads(None, None)
    if mN == 0.0:
        raise ValueError("the norm network is zero")
    E = 0.0
    acc = [ftn.axpy(-1.0, gN[s], gN[s]) for s in range(n)]  # zero tensors of the ket structures
    parts = []
    for G, sites in terms:
        m, e, g = value_and_ket_grads(G, tuple(sites))
        w = 2.0 ** (e - eN) / mN            # dX_t / N in units of the returned gradients
        E += m * 2.0 ** (e - eN) / mN
        parts.append((w, g))
    for w, g in parts:
        for s in range(n):
            acc[s] = ftn.axpy(w, g[s], acc[s])
    # - E dN / N
    for s in range(n):
        acc[s] = ftn.axpy(-E / mN, gN[s], acc[s])
    return E, acc
