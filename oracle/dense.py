"""Brute-force definitions of a fermionic network's value (pins for tests).

``koszul_value`` (global convention, Sec. II.D): list every leg of every
tensor in position order. For one assignment of indices to all bonds and
open legs, the term is the product of entries times (-1)^kappa, where kappa
is the Koszul sign (sum of p_x p_y over inverted pairs) of the permutation
taking that flat list to [open legs in flat order] ++ [the two ends of each
bond, side by side]. Bond pairs are even, so where they stand does not
matter. Summing over all assignments gives the network value. In the local
convention (Sec. II.E) the value for a chosen tensor order is the same sum
with the bond parity (-1)^{p_e} for every bond whose '+' end (arrow tail) is
on the earlier tensor, i.e. that is contracted against its arrow.

``swap_gate_value`` (the older method of Sec. I: a bosonic network with
swap tensors inserted by hand) for closed networks: with all legs on a line
in flat order and every bond drawn as an arc between its ends, each pair of
arcs whose ends interleave crosses once and contributes a swap gate
(-1)^{p p'}; nested or disjoint arcs contribute nothing.

Both routes build one dense ``numpy.einsum`` and share nothing with
``ops``/``network``.
"""

import numpy as np

from . import symmetry as S


def leg_parity_vector(sym, leg):
    out = []
    for q, d in zip(leg.charges, leg.dims):
        out += [S.parity(sym, q)] * d
    return np.array(out, dtype=np.int64)


def _einsum_value(operands):
    args = []
    for arr, idx in operands:
        args.append(arr)
        args.append(list(idx))
    return args


def koszul_value(tensors, bonds, order, local=False, open_legs=None):
    """Dense value of a network by the Koszul definition.

    ``tensors``: dict id -> FTensor; ``bonds``: (t1, l1, t2, l2);
    ``order``: tensor ids in global order. Open legs are returned as axes in
    flat order. With ``local=True`` the local-convention bond parity is
    included for the given order.
    """
    sym = next(iter(tensors.values())).sym
    flat = [(t, l) for t in order for l in range(tensors[t].ndim)]
    fpos = {fl: i for i, fl in enumerate(flat)}
    var = {}
    pairs = []
    for bi, (t1, l1, t2, l2) in enumerate(bonds):
        a, b = fpos[(t1, l1)], fpos[(t2, l2)]
        if a > b:
            a, b = b, a
        var[a] = ("b", bi)
        var[b] = ("b", bi)
        pairs.append((a, b))
    opens = [i for i in range(len(flat)) if i not in var]
    for i in opens:
        var[i] = ("o", i)
    target = list(opens)
    for a, b in pairs:
        target += [a, b]
    tpos = {f: k for k, f in enumerate(target)}
    # parity vector per variable
    vnames = sorted(set(var.values()), key=str)
    vid = {v: k for k, v in enumerate(vnames)}
    pvec = {}
    dim = {}
    for i, (t, l) in enumerate(flat):
        leg = tensors[t].legs[l]
        pv = leg_parity_vector(sym, leg)
        v = vid[var[i]]
        if v in pvec:
            if dim[v] != leg.size or not np.array_equal(pvec[v], pv):
                raise ValueError("bond ends with different index spaces")
        pvec[v] = pv
        dim[v] = leg.size
    # pairwise sign counts
    cnt = {}
    n = len(flat)
    for x in range(n):
        for y in range(x + 1, n):
            if tpos[x] > tpos[y]:
                u, w = vid[var[x]], vid[var[y]]
                key = (min(u, w), max(u, w))
                cnt[key] = cnt.get(key, 0) ^ 1
    if local:
        for bi, (t1, l1, t2, l2) in enumerate(bonds):
            first = (t1, l1) if fpos[(t1, l1)] < fpos[(t2, l2)] else (t2, l2)
            if tensors[first[0]].legs[first[1]].dual == 0:
                v = vid[("b", bi)]
                cnt[(v, v)] = cnt.get((v, v), 0) ^ 1
    ops = []
    for t in order:
        idx = [vid[var[fpos[(t, l)]]] for l in range(tensors[t].ndim)]
        ops.append((tensors[t].to_dense(), idx))
    for (u, w), c in cnt.items():
        if not c:
            continue
        if u == w:
            ops.append(((-1.0) ** pvec[u], [u]))
        else:
            ops.append(((-1.0) ** np.outer(pvec[u], pvec[w]), [u, w]))
    out_idx = [vid[var[i]] for i in opens]
    args = _einsum_value(ops)
    args.append(out_idx)
    return np.einsum(*args, optimize="greedy")


def swap_gate_value(tensors, bonds, order):
    """Closed-network value as a bosonic network with swap gates.

    Legs on a line in flat order; bond e is the arc between its two ends.
    Two arcs (a, b) and (c, d) with a < c cross iff a < c < b < d; each
    crossing is a swap gate (-1)^{p_e p_f}. For a closed network of
    tensors in one order, the value is the plain contraction with every
    crossing's gate inserted (and no other sign).
    """
    sym = next(iter(tensors.values())).sym
    flat = [(t, l) for t in order for l in range(tensors[t].ndim)]
    fpos = {fl: i for i, fl in enumerate(flat)}
    arcs = []
    for bi, (t1, l1, t2, l2) in enumerate(bonds):
        a, b = fpos[(t1, l1)], fpos[(t2, l2)]
        arcs.append((min(a, b), max(a, b), bi))
    if len(arcs) * 2 != len(flat):
        raise ValueError("swap_gate_value needs a closed network")
    pv = {}
    for bi, (t1, l1, t2, l2) in enumerate(bonds):
        pv[bi] = leg_parity_vector(sym, tensors[t1].legs[l1])
    ops = []
    for t in order:
        idx = []
        for l in range(tensors[t].ndim):
            f = fpos[(t, l)]
            bi = next(b for (a, c, b) in arcs if a == f or c == f)
            idx.append(bi)
        ops.append((tensors[t].to_dense(), idx))
    for i, (a, b, e) in enumerate(arcs):
        for (c, d, f) in arcs[i + 1:]:
            if (a < c < b < d) or (c < a < d < b):
                ops.append(((-1.0) ** np.outer(pv[e], pv[f]), [e, f]))
    args = _einsum_value(ops)
    args.append([])
    return float(np.einsum(*args, optimize="greedy"))
