"""Reverse-mode derivatives of the oracle's contractions (test infrastructure).

A pairwise contraction is bilinear in its two operands (Eq.
standardcontract: every output entry is a signed sum of products of one
entry of each), and the value of a closed network is linear in each of its
tensors (Eqs. fermionictn, fermionictn2). The derivatives below are obtained
by torch's reverse-mode differentiation of the oracle's own block arithmetic
(``ops.ftensordot``, ``network.contract_network`` with no truncation), so
they inherit its signs: nothing is re-derived here.

* ``ftensordot_vjp``: cotangents (dA, dB) of C = ftensordot(A, B) for a
  given output cotangent dC, i.e. the gradients of <dC, C>.
* ``network_grad``: value of a closed network and its gradient with respect
  to every allowed entry of every tensor.
* ``compress_product_grad``: gradient of <W, F(A'B')> through bond
  compression (Sec. II.A truncated SVD, kept counts fixed); the compressed
  factors are differentiated through the SVD of the bond matrix itself.
"""

import torch

from .tensor import FTensor
from .ops import ftensordot
from .network import Network, contract_network


def _leaf_copy(T):
    out = FTensor(T.sym, T.legs, T.total)
    for k in T.keys():
        out.blocks[k] = T.block(k).detach().clone().requires_grad_(True)
    return out


def inner(X, Y):
    """<X, Y> = sum over common blocks of the entrywise products."""
    s = 0.0
    for k in X.keys():
        if k in Y.blocks:
            s = s + (X.block(k) * Y.block(k)).sum()
    return s


def ftensordot_vjp(A, B, dC, axes_a, axes_b, conv="local"):
    """(dA, dB) = gradients of <dC, ftensordot(A, B, axes_a, axes_b)>."""
    A1, B1 = _leaf_copy(A), _leaf_copy(B)
    C = ftensordot(A1, B1, axes_a, axes_b, conv=conv)
    L = inner(dC, C)
    if not torch.is_tensor(L) or not L.requires_grad:
        return FTensor.zeros(A.sym, A.legs, A.total), FTensor.zeros(B.sym, B.legs, B.total)
    leaves = [A1, B1]
    keys = [T.keys() for T in leaves]
    flat = [T.blocks[k] for T, ks in zip(leaves, keys) for k in ks]
    gs = torch.autograd.grad(L, flat, allow_unused=True) if flat else []
    outs, i = [], 0
    for T, ks in zip(leaves, keys):
        o = FTensor(T.sym, T.legs, T.total)
        for k in ks:
            g = gs[i]
            o.blocks[k] = torch.zeros_like(T.blocks[k].detach()) if g is None else g.detach()
            i += 1
        outs.append(o)
    return outs[0], outs[1]


def network_grad(net, path, chi=None):
    """(value, {tensor id: gradient FTensor}) of a closed network, exact or
    approximate (compression as early as possible, kept counts fixed)."""
    leaves = {t: _leaf_copy(x) for t, x in net.tensors.items()}
    net2 = Network(leaves, net.bonds, conv=net.conv, positions=net.positions)
    T, labs, e, _ = contract_network(net2, path, chi=chi, renorm=False)
    if T.ndim != 0:
        raise ValueError("network is not closed")
    b = T.blocks.get(())
    ids = sorted(leaves)
    flat = [leaves[t].blocks[k] for t in ids for k in leaves[t].keys()]
    if b is None or not b.requires_grad:
        gs = [None] * len(flat)
    else:
        gs = torch.autograd.grad(b.sum(), flat, allow_unused=True)
    grads, i = {}, 0
    for t in ids:
        o = FTensor(leaves[t].sym, leaves[t].legs, leaves[t].total)
        for k in leaves[t].keys():
            g = gs[i]
            o.blocks[k] = torch.zeros_like(leaves[t].blocks[k].detach()) if g is None else g.detach()
            i += 1
        grads[t] = o
    return (0.0 if b is None else float(b.detach())), grads


def compress_product_grad(A, B, la, lb, chi, W, conv="local", cutoff=1e-6):
    """(dA, dB) = gradients of <W, F(A' B')> over the bond, for
    (A', B') = compress_bond(A, B, ...): a loss that does not depend on the
    sign chosen for each kept singular vector pair, taken in one reverse-mode
    pass through the oracle's truncated SVD (kept counts fixed)."""
    from .linalg import compress_bond
    A1, B1 = _leaf_copy(A), _leaf_copy(B)
    A2, B2, _ = compress_bond(A1, B1, la, lb, chi, conv=conv, cutoff=cutoff)
    L = inner(W, ftensordot(A2, B2, [la], [lb], conv=conv))
    leaves = [A1, B1]
    flat = [T.blocks[k] for T in leaves for k in T.keys()]
    ok = flat and torch.is_tensor(L) and L.requires_grad
    gs = torch.autograd.grad(L, flat, allow_unused=True) if ok else [None] * len(flat)
    outs, i = [], 0
    for T in leaves:
        o = FTensor(T.sym, T.legs, T.total)
        for k in T.keys():
            g = gs[i]
            o.blocks[k] = torch.zeros_like(T.blocks[k].detach()) if g is None else g.detach()
            i += 1
        outs.append(o)
    return outs[0], outs[1]


def energy_grad(spec, kets, terms, paths, chi=None):
    """(E, [dE/dket_s]) for E = sum_t <psi|G_t|psi> / <psi|psi>.

    ``terms``: list of (G FTensor, (u, v)); ``paths``: {None: norm path,
    (u, v): term path}. Every network is contracted (approximately with
    chi) by ``network.contract_network`` in the local convention; the bra
    tensors are the daggers of the kets, so both layers carry the gradient.
    """
    from .physics import norm_network
    leaves = [_leaf_copy(k) for k in kets]

    def value(op=None, sites=None):
        net = norm_network(spec, leaves, op=op, op_sites=sites, conv="local")
        T, _, e, _ = contract_network(net, paths[None if op is None else tuple(sites)], chi=chi, renorm=False)
        b = T.blocks.get(())
        return (b if b is not None else torch.zeros((), dtype=torch.float64)) * 2.0 ** e

    N = value()
    E = sum(value(G, s) for G, s in terms) / N
    flat = [T.blocks[k] for T in leaves for k in T.keys()]
    gs = torch.autograd.grad(E, flat, allow_unused=True)
    out, i = [], 0
    for T in leaves:
        o = FTensor(T.sym, T.legs, T.total)
        for k in T.keys():
            g = gs[i]
            o.blocks[k] = torch.zeros_like(T.blocks[k].detach()) if g is None else g.detach()
            i += 1
        out.append(o)
    return float(E.detach()), out
