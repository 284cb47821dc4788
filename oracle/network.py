"""Network contraction along an SSA path, exact and approximate.

Two conventions, each implemented as the paper describes it:

* Global (Sec. II.D, Eq. fermionictn): every tensor has a position and the
  value is F(T^[0] T^[1] ...). To contract X and Y (X earlier), Y is moved
  left past each tensor Z in between: every bond Y shares with Z gets the
  bond parity on Y's leg and odd Y, Z give the phase (-1)^{p(Y)p(Z)} (the
  swap rule, Eq. fermiswap). Then X and Y are adjacent and contracted with
  the global convention; the result takes X's position.
* Local (Sec. II.E, Eq. fermionictn2): arrows live on bonds (duals); every
  contraction is a pairwise local ``ftensordot``. Odd tensors receive a
  size-1 odd dummy leg in front; at the end the dummies are sorted by the
  chosen global order of their tensors and the phase (-1)^{m(m-1)/2} of
  having prepended them is removed.

Approximate contraction (Fig. 1b, Sec. III, compression as early as
possible): after each pairwise contraction the bonds the new tensor shares
with one neighbour are fused into one bond (Sec. IV.A), and every such bond
larger than chi is compressed with ``compress_bond`` (singular values not
above 1e-12 of the largest count as zero). Each intermediate is
rescaled by a power of two, accumulated in an integer exponent (exact in
binary floating point).
"""

import math

import torch

from . import symmetry as S
from .ops import (ftensordot, ftranspose, leg_parity_sign, fuse, add_dummy,
                  flip_dual, koszul)
from .linalg import compress_bond


class Network:
    """Tensors keyed by id plus bonds ``(t1, l1, t2, l2)``.

    ``positions``: optional global position of every tensor id (list indexed
    by id). ``conv``: "global" or "local". Open legs are those in no bond.
    """

    def __init__(self, tensors, bonds, conv="local", positions=None):
        self.tensors = dict(enumerate(tensors)) if isinstance(tensors, list) else dict(tensors)
        self.bonds = [tuple(b) for b in bonds]
        self.conv = conv
        self.positions = None if positions is None else list(positions)


class _State:
    def __init__(self, net):
        self.T = {t: x for t, x in net.tensors.items()}
        # leg labels: for each tensor, list of label per leg; label is
        # ('b', bond_id, end) for bonded legs, ('o', tensor, leg) for open
        self.lab = {}
        for t, x in self.T.items():
            self.lab[t] = [("o", t, l) for l in range(x.ndim)]
        self.bond_end = {}
        for bi, (t1, l1, t2, l2) in enumerate(net.bonds):
            self.lab[t1][l1] = ("b", bi)
            self.lab[t2][l2] = ("b", bi)
        self.nbid = len(net.bonds)
        self.exp2 = 0


def _shared(st, x, y):
    lx, ly = [], []
    for i, lab in enumerate(st.lab[x]):
        if lab[0] == "b" and lab in st.lab[y]:
            lx.append(i)
            ly.append(st.lab[y].index(lab))
    # order pairs by bond id
    pairs = sorted(zip(lx, ly), key=lambda p: st.lab[x][p[0]][1])
    return [p[0] for p in pairs], [p[1] for p in pairs]


def _renorm(st, z):
    m = st.T[z].max_abs()
    if m > 0 and math.isfinite(m):
        e = math.frexp(m)[1]
        st.T[z] = st.T[z].scaled(2.0 ** (-e))
        st.exp2 += e


def _neighbours(st, z):
    out = {}
    for i, lab in enumerate(st.lab[z]):
        if lab[0] != "b":
            continue
        for t, labs in st.lab.items():
            if t != z and lab in labs:
                out.setdefault(t, []).append(i)
    return out


# relative singular-value cutoff of network compression: values not above
# 1e-12 of the largest are numerically zero (the FP64 round-off of an SVD is
# ~1e-15 of the largest); the paper keeps the chi largest values and names
# no cutoff
CUTOFF = 1e-12


def _fuse_and_compress(st, z, chi, conv, order, cutoff=CUTOFF):
    """Fuse parallel bonds of z to each neighbour, then compress > chi."""
    infos = []
    for w in sorted(_neighbours(st, z)):
        lz = _neighbours(st, z)[w]
        lz = sorted(lz, key=lambda i: st.lab[z][i][1])
        lw = [st.lab[w].index(st.lab[z][i]) for i in lz]
        if len(lz) > 1:
            if conv == "local":
                Z2, _ = fuse(st.T[z], lz, conv="local")
                W2, _ = fuse(st.T[w], lw, conv="local")
            else:
                z_later = order.index(z) > order.index(w)
                Z2, _ = fuse(st.T[z], lz, conv="global", rev=z_later)
                W2, _ = fuse(st.T[w], lw, conv="global", rev=not z_later)
            bid = st.nbid
            st.nbid += 1
            for T_, t_, ls in ((Z2, z, lz), (W2, w, lw)):
                rest = [lab for i, lab in enumerate(st.lab[t_]) if i not in ls]
                pos = sum(1 for i in range(st.T[t_].ndim) if i not in ls and i < ls[0])
                st.lab[t_] = rest[:pos] + [("b", bid)] + rest[pos:]
                st.T[t_] = T_
            lz = [st.lab[z].index(("b", bid))]
            lw = [st.lab[w].index(("b", bid))]
        dim = st.T[z].legs[lz[0]].size
        # a tensor with no allowed block is exactly zero: every later product
        # vanishes and there is no spectrum to truncate, so the bond is kept
        empty = st.T[z].nnz() == 0 or st.T[w].nnz() == 0
        if chi is not None and dim > chi and not empty:
            if conv == "local":
                A, B, info = compress_bond(st.T[z], st.T[w], lz[0], lw[0], chi, conv="local", cutoff=cutoff)
                st.T[z], st.T[w] = A, B
            else:
                if order.index(z) < order.index(w):
                    A, B, info = compress_bond(st.T[z], st.T[w], lz[0], lw[0], chi, conv="global",
                                               cutoff=cutoff)
                    st.T[z], st.T[w] = A, B
                else:
                    A, B, info = compress_bond(st.T[w], st.T[z], lw[0], lz[0], chi, conv="global",
                                               cutoff=cutoff)
                    st.T[w], st.T[z] = A, B
            infos.append(info)
    return infos


def contract_network(net, path, chi=None, renorm=True, dummy_order=None):
    """Contract ``net`` along an SSA ``path``.

    Returns ``(T, labels, exp2, infos)``: the final tensor (a scalar tensor
    if the network is closed), the original ``(tensor, leg)`` of each of its
    legs (dummy legs are labelled ``('d', tensor)``), the accumulated
    power-of-two exponent and the compression infos. In the local convention
    dummy legs have already been sorted and removed, and ``labels`` lists
    only the open legs.
    """
    conv = net.conv
    st = _State(net)
    infos = []
    if conv == "global":
        if net.positions is None:
            raise ValueError("global convention needs positions")
        order = sorted(st.T, key=lambda t: net.positions[t])
    else:
        order = sorted(st.T)
        if dummy_order is None:
            dummy_order = net.positions
        dummy_rank = {}
        dord = sorted(st.T, key=(lambda t: dummy_order[t]) if dummy_order is not None else (lambda t: t))
        for t in list(st.T):
            if st.T[t].parity:
                st.T[t] = add_dummy(st.T[t])
                st.lab[t] = [("d", t)] + st.lab[t]
        for r, t in enumerate([t for t in dord if st.lab[t] and st.lab[t][0] == ("d", t)]):
            dummy_rank[t] = r
    ssa = {i: t for i, t in enumerate(sorted(st.T))}
    nid = max(st.T) + 1
    for (i, j) in path:
        x, y = ssa[i], ssa[j]
        if conv == "global":
            if order.index(x) > order.index(y):
                x, y = y, x
            px, py = order.index(x), order.index(y)
            Y = st.T[y]
            for z in order[px + 1:py]:
                # bonds shared by Y and Z get the bond parity on Y's legs
                for li, lab in enumerate(st.lab[y]):
                    if lab[0] == "b" and lab in st.lab[z]:
                        Y = leg_parity_sign(Y, li)
                if Y.parity and st.T[z].parity:
                    Y = Y.scaled(-1.0)
            st.T[y] = Y
        lx, ly = _shared(st, x, y)
        Z = ftensordot(st.T[x], st.T[y], lx, ly, conv=conv)
        z = nid
        nid += 1
        st.T[z] = Z
        st.lab[z] = ([l for k, l in enumerate(st.lab[x]) if k not in lx] +
                     [l for k, l in enumerate(st.lab[y]) if k not in ly])
        if conv == "global":
            k = order.index(x)
            order[k] = z
            order.remove(y)
        for t in (x, y):
            del st.T[t]
            del st.lab[t]
        ssa[len(ssa)] = z
        if chi is not None:
            infos += _fuse_and_compress(st, z, chi, conv, order)
        if renorm:
            _renorm(st, z)
    if len(st.T) != 1:
        raise ValueError("path does not contract the network to one tensor")
    (z, T), = st.T.items()
    labs = st.lab[z]
    if conv == "local":
        dpos = [k for k, l in enumerate(labs) if l[0] == "d"]
        m = len(dpos)
        if m:
            others = [k for k in range(T.ndim) if k not in dpos]
            dsorted = sorted(dpos, key=lambda k: dummy_rank[labs[k][1]])
            T = ftranspose(T, dsorted + others)
            # remove the dummy legs (size 1) and the prepending phase
            sgn = -1.0 if (m * (m - 1) // 2) % 2 else 1.0
            T = _drop_leading_dummies(T, m).scaled(sgn)
            labs = [labs[k] for k in others]
    return T, labs, st.exp2, infos


def _drop_leading_dummies(T, m):
    from .tensor import FTensor
    sym = T.sym
    tot = T.total
    for l in T.legs[:m]:
        tot = S.add(sym, tot, S.neg(sym, S.signed(sym, l.dual, l.charges[0])))
    out = FTensor(sym, T.legs[m:], tot)
    for key in T.keys():
        out.blocks[key[m:]] = T.block(key).reshape(T.block(key).shape[m:]).clone()
    return out


def scalar_value(T):
    """The single entry of a 0-leg tensor (0.0 if its block is not allowed)."""
    if T.ndim != 0:
        raise ValueError("not a scalar")
    b = T.blocks.get(())
    return 0.0 if b is None else float(b)


def network_value(net, path, chi=None):
    """Scalar value of a closed network as (mantissa, exp2)."""
    T, labs, e, _ = contract_network(net, path, chi=chi)
    return scalar_value(T), e


def to_local(net):
    """Re-express a global-convention network in the local convention.

    Sec. II.D: a global order is a DAG whose arrows point from later to
    earlier tensors, and working with positions is equivalent to working
    with that DAG. In the local convention the arrows are read from the
    duals, so every bond whose '-' end sits on the later tensor has both
    ends' duals flipped (with conjugated charges). In the global convention
    duals only label charges, so this relabelling changes no value and
    inserts no sign. Dummy legs of odd tensors are sorted by position.
    """
    pos = net.positions
    T = {t: x for t, x in net.tensors.items()}
    for (t1, l1, t2, l2) in net.bonds:
        # the '-' end is the arrow head; it must be on the earlier tensor
        head = t1 if T[t1].legs[l1].dual == 1 else t2
        other = t2 if head == t1 else t1
        if pos[head] > pos[other]:
            T[t1] = flip_dual(T[t1], l1, with_sign=False)
            T[t2] = flip_dual(T[t2], l2, with_sign=False)
    return Network(T, net.bonds, conv="local", positions=pos)
