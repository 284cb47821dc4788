"""Fermionic tensor operations, written from their definitions.

* ``ftranspose``: Eq. (transposition) gives (-1)^{p_i p_j} for swapping two
  adjacent legs; a general permutation is a product of adjacent swaps, so
  the sign is the sum, over every pair of legs whose relative order the
  permutation inverts, of p_i p_j (mod 2).
* ``ftensordot``: Eq. (standardcontract): move the contracted legs of A to
  its end and those of B to its front (fermionic transpositions), then
  contract them pairwise. Pairs are formed by list position (a_t, b_t); the
  sign-free arrangement is the mirror one (a_1..a_k, b_k..b_1), so listing B's
  legs in the same order as A's costs the reversal sign sum_{s<t} p_s p_t,
  the rule Sec. IV.A states for a fused inward bond.
* Conventions: ``conv="global"`` is F(AB) with A immediately left of B
  (Sec. II.D). ``conv="local"`` (Sec. II.E) reads arrows from the duals (an
  arrow runs from the '+' end to the '-' end, Sec. IV.B): a bond whose '-'
  end (the arrow head) is on the left tensor is contracted along the arrow
  and costs nothing; otherwise the bond parity (-1)^{p} is applied.
* ``flip_dual``: reversing an arrow is equivalent to a bond parity tensor
  (Sec. II.E, Fig. 3b). One end of a bond is flipped with the parity sign,
  the other without; this module puts the sign on the end that was '-', so
  flipping both ends of a bond reverses it and inserts exactly one g.
* ``fuse``: the three parity contributions of Sec. IV.A.
"""

import itertools

import numpy as np
import torch

from . import symmetry as S
from .tensor import FTensor, Leg, make_leg


def koszul(parities, perm):
    """Sign exponent of reordering legs: new position t holds old leg perm[t]."""
    s = 0
    n = len(perm)
    for t in range(n):
        for u in range(t + 1, n):
            if perm[t] > perm[u]:
                s ^= parities[perm[t]] & parities[perm[u]]
    return s


def ftranspose(T, perm):
    perm = [int(p) for p in perm]
    if sorted(perm) != list(range(T.ndim)):
        raise ValueError("not a permutation")
    legs = [T.legs[p] for p in perm]
    out = FTensor(T.sym, legs, T.total)
    for key in T.keys():
        par = T.key_parities(key)
        sgn = -1.0 if koszul(par, perm) else 1.0
        nk = tuple(key[p] for p in perm)
        b = T.block(key)
        out.blocks[nk] = sgn * (b.permute(*perm) if perm else b)
    return out


def leg_parity_sign(T, leg):
    """Multiply every block by (-1)^{p} of its sector on ``leg`` (a g tensor)."""
    out = FTensor(T.sym, T.legs, T.total)
    for key in T.keys():
        p = S.parity(T.sym, T.legs[leg].charges[key[leg]])
        out.blocks[key] = -T.block(key) if p else T.block(key).clone()
    return out


def flip_dual(T, leg, with_sign=None):
    """Reverse the dual of one leg; charges are conjugated so the blocks stay.

    ``with_sign`` defaults to "the leg was '-'" (see module docstring).
    """
    old = T.legs[leg]
    if with_sign is None:
        with_sign = bool(old.dual)
    sym = T.sym
    newleg = make_leg(sym, [S.neg(sym, q) for q in old.charges], old.dims, 1 - old.dual)
    remap = [newleg.index_of(S.neg(sym, q)) for q in old.charges]
    legs = list(T.legs)
    legs[leg] = newleg
    out = FTensor(sym, legs, T.total)
    for key in T.keys():
        nk = list(key)
        nk[leg] = remap[key[leg]]
        b = T.block(key)
        neg_it = with_sign and S.parity(sym, old.charges[key[leg]])
        out.blocks[tuple(nk)] = -b if neg_it else b.clone()
    return out


def _check_pair(sym, la, lb):
    if la.dual == lb.dual:
        raise ValueError("contracted legs must have opposite duals")
    for q, d in zip(la.charges, la.dims):
        db = lb.dim_of(q)
        if db and db != d:
            raise ValueError("sector dimension mismatch on a contracted bond")


def ftensordot(A, B, axes_a, axes_b, conv="local"):
    """Fermionic contraction, output legs = free(A) ++ free(B)."""
    if A.sym != B.sym:
        raise ValueError("symmetry mismatch")
    sym = A.sym
    axes_a = [int(a) for a in axes_a]
    axes_b = [int(b) for b in axes_b]
    k = len(axes_a)
    if k != len(axes_b):
        raise ValueError("axes length mismatch")
    for a, b in zip(axes_a, axes_b):
        _check_pair(sym, A.legs[a], B.legs[b])
    free_a = [i for i in range(A.ndim) if i not in axes_a]
    free_b = [i for i in range(B.ndim) if i not in axes_b]
    At = ftranspose(A, free_a + axes_a)
    Bt = ftranspose(B, axes_b + free_b)
    na = len(free_a)
    legs = list(At.legs[:na]) + list(Bt.legs[k:])
    C = FTensor.zeros(sym, legs, S.add(sym, A.total, B.total))
    plus_on_left = [A.legs[a].dual == 0 for a in axes_a]
    for ka in At.keys():
        qa = At.key_charges(ka)[na:]
        for kb in Bt.keys():
            qb = Bt.key_charges(kb)[:k]
            if qa != qb:
                continue
            ps = [S.parity(sym, q) for q in qb]
            e = 0
            for s in range(k):
                for t in range(s + 1, k):
                    e ^= ps[s] & ps[t]
            if conv == "local":
                for t in range(k):
                    if plus_on_left[t]:
                        e ^= ps[t]
            elif conv != "global":
                raise ValueError("conv must be 'local' or 'global'")
            prod = torch.tensordot(At.block(ka), Bt.block(kb),
                                   dims=(list(range(na, na + k)), list(range(k))))
            key = tuple(ka[:na]) + tuple(kb[k:])
            C.blocks[key] = C.blocks[key] + (-prod if e else prod)
    return C


def dagger(T):
    """Hermitian conjugate of one tensor: legs reversed, duals flipped.

    The reversal is a relabelling with no Koszul sign; charges keep their
    labels and the total charge is negated. Entries are real here.
    """
    sym = T.sym
    legs = [Leg(l.charges, l.dims, 1 - l.dual) for l in reversed(T.legs)]
    out = FTensor(sym, legs, S.neg(sym, T.total))
    n = T.ndim
    for key in T.keys():
        b = T.block(key)
        out.blocks[tuple(reversed(key))] = (b.permute(*reversed(range(n))) if n else b).clone()
    return out


def add_dummy(T):
    """Prepend a size-1 odd leg ('+') making an odd tensor even (Sec. II.E)."""
    sym = T.sym
    qd = S.neg(sym, T.total)
    if S.parity(sym, qd) != 1:
        raise ValueError("add_dummy needs an odd tensor")
    leg = Leg((qd,), (1,), 0)
    out = FTensor(sym, (leg,) + T.legs, S.zero(sym))
    for key in T.keys():
        out.blocks[(0,) + key] = T.block(key).unsqueeze(0).clone()
    return out


class FuseInfo:
    """How a fused leg decomposes: original legs and sub-combination offsets."""

    def __init__(self, legs, fused_leg, table):
        self.legs = legs          # the component legs after dual alignment
        self.fused_leg = fused_leg
        self.table = table        # component key tuple -> (fused sector, offset)


def _fused_leg(sym, comp_legs):
    dual = comp_legs[0].dual
    combos = {}
    for key in itertools.product(*[range(l.nsect) for l in comp_legs]):
        q = S.zero(sym)
        d = 1
        for l, i in zip(comp_legs, key):
            q = S.add(sym, q, l.charges[i])
            d *= l.dims[i]
        combos.setdefault(q, []).append((key, d))
    charges = sorted(combos)
    dims = []
    table = {}
    for si, q in enumerate(charges):
        off = 0
        for key, d in sorted(combos[q]):
            table[key] = (si, off)
            off += d
        dims.append(off)
    return Leg(tuple(charges), tuple(dims), dual), table


def fuse(T, legs, conv="local", rev=None):
    """Fuse ``legs`` (in the given order) into one leg (Sec. IV.A).

    The fused leg takes the place of ``legs[0]`` among the remaining legs.
    Steps: (1) fermionic transposition making the legs adjacent; (2) legs
    whose dual differs from the first are flipped (``flip_dual``; in the
    global convention arrows come from positions, so the flip is a pure
    relabelling without sign); (3) the reversal sign sum_{s<t} p_s p_t is
    applied if the fused bond is inward ('-') in the local convention, or if
    ``rev`` is true in the global convention (the later of the two tensors
    sharing the bond carries it).
    """
    sym = T.sym
    legs = [int(l) for l in legs]
    rest = [i for i in range(T.ndim) if i not in legs]
    pos = sum(1 for i in rest if i < legs[0])
    order = rest[:pos] + legs + rest[pos:]
    X = ftranspose(T, order)
    m = len(legs)
    d0 = X.legs[pos].dual
    for j in range(pos + 1, pos + m):
        if X.legs[j].dual != d0:
            X = flip_dual(X, j, with_sign=(None if conv == "local" else False))
    if conv == "local":
        do_rev = d0 == 1
    else:
        do_rev = bool(rev)
    comp = list(X.legs[pos:pos + m])
    fleg, table = _fused_leg(sym, comp)
    newlegs = list(X.legs[:pos]) + [fleg] + list(X.legs[pos + m:])
    out = FTensor.zeros(sym, newlegs, X.total)
    for key in X.keys():
        b = X.block(key)
        ck = tuple(key[pos:pos + m])
        ps = [S.parity(sym, comp[j].charges[ck[j]]) for j in range(m)]
        e = 0
        if do_rev:
            for s in range(m):
                for t in range(s + 1, m):
                    e ^= ps[s] & ps[t]
        si, off = table[ck]
        nk = tuple(key[:pos]) + (si,) + tuple(key[pos + m:])
        shp = list(b.shape)
        sub = int(np.prod(shp[pos:pos + m])) if m else 1
        flat = b.reshape(shp[:pos] + [sub] + shp[pos + m:])
        tgt = out.blocks[nk]
        idx = [slice(None)] * len(newlegs)
        idx[pos] = slice(off, off + sub)
        tgt = tgt.clone()
        tgt[tuple(idx)] = -flat if e else flat
        out.blocks[nk] = tgt
    return out, FuseInfo(comp, fleg, table)


def tensordot_bosonic(A, B, axes_a, axes_b):
    """Plain block contraction without any sign (the bosonic case, Sec. II.C)."""
    sym = A.sym
    free_a = [i for i in range(A.ndim) if i not in axes_a]
    free_b = [i for i in range(B.ndim) if i not in axes_b]
    legs = [A.legs[i] for i in free_a] + [B.legs[i] for i in free_b]
    C = FTensor.zeros(sym, legs, S.add(sym, A.total, B.total))
    for ka in A.keys():
        for kb in B.keys():
            if [A.legs[a].charges[ka[a]] for a in axes_a] != [B.legs[b].charges[kb[b]] for b in axes_b]:
                continue
            prod = torch.tensordot(A.block(ka), B.block(kb), dims=(list(axes_a), list(axes_b)))
            key = tuple(ka[i] for i in free_a) + tuple(kb[i] for i in free_b)
            C.blocks[key] = C.blocks[key] + prod
    return C
