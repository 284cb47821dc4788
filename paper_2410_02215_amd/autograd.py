"""Reverse-mode derivatives of fermionic contractions on the GPU.

``dot`` is a differentiable ``ftensordot``. Its backward pass calls
``ftn_ftensordot_backward``: the contraction of Eq. (standardcontract) is
bilinear, so with the signed fused matrices A~, B~ of the forward pass the
cotangents are dA~ = dC B~^T and dB~ = A~^T dC per fused charge, returned to
the block layouts by the inverse signed permutes. ``transpose`` is a
differentiable ``ftranspose``: a signed permutation is orthogonal, so its
adjoint is the inverse permutation with the same signs.

``compress`` is a differentiable ``compress_bond`` through
``ftn_compress_bond_backward`` (the truncated-SVD derivative).

``contract_exact`` contracts a network in the local convention (Sec. II.E,
Eq. fermionictn2) along an SSA path with these operations, so that
``torch.autograd`` differentiates the network value with respect to the
block data of every tensor. Odd tensors receive a size-1 odd dummy leg in
front (it changes no block data); at the end the dummies are sorted by the
chosen global order of their tensors, dropped, and the phase (-1)^{m(m-1)/2}
of having prepended m of them is removed. Shared bonds of a step are paired
in increasing bond order. Every step runs in the HIP library; torch only
holds the block data and records the graph.
"""

import torch

from . import ftn


def _neg(sym, q):
    return ((-q[0]) % 2, 0) if sym == ftn.Z2 else (-q[0], -q[1] if sym == ftn.U1xU1 else 0)


def _parity(sym, q):
    return (q[0] + (q[1] if sym == ftn.U1xU1 else 0)) % 2


def _sub(sym, a, b):
    if sym == ftn.Z2:
        return ((a[0] - b[0]) % 2, 0)
    return (a[0] - b[0], a[1] - b[1] if sym == ftn.U1xU1 else 0)


class DTensor:
    """Block data (1-D torch device tensor, may require grad) plus structure.

    ``legs``: list of (charges, dims, dual) as taken by ``ftn.Tensor.create``;
    ``total``: the total charge as a pair.
    """

    def __init__(self, sym, legs, total, data):
        self.sym = int(sym)
        self.legs = [([tuple(q) for q in c], [int(x) for x in d], int(u)) for (c, d, u) in legs]
        self.total = tuple(int(x) for x in total)
        self.data = data

    @property
    def dtype(self):
        return ftn.F64 if self.data.dtype == torch.float64 else ftn.F32

    @property
    def ndim(self):
        return len(self.legs)

    @property
    def parity(self):
        return _parity(self.sym, self.total)

    def handle(self, data=None):
        """An ftn.Tensor over ``data`` (default: the current data) without a
        copy (ftn_tensor_wrap); the wrapper keeps the torch tensor alive."""
        d = (self.data if data is None else data).detach().contiguous()
        return ftn.Tensor.wrap(self.sym, self.legs, self.total, d)

    @classmethod
    def from_tensor(cls, t, requires_grad=False):
        inf = t.info()
        data = t.data()
        if requires_grad:
            data.requires_grad_(True)
        return cls(inf["sym"], t.legs(), inf["total"], data)


class _Dot(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_data, b_data, a, b, axes_a, axes_b, conv, gemm, out):
        A, B = a.handle(a_data), b.handle(b_data)
        C = ftn.ftensordot(A, B, axes_a, axes_b, conv, gemm)
        inf = C.info()
        out.append((C.legs(), inf["total"]))
        ctx.A, ctx.B = A, B
        ctx.args = (axes_a, axes_b, conv, gemm, a.sym, C.legs(), inf["total"], a.dtype)
        return C.data_view()

    @staticmethod
    def backward(ctx, dc):
        axes_a, axes_b, conv, gemm, sym, legs, total, dtype = ctx.args
        DC = ftn.Tensor.create(sym, legs, total, dtype, data=dc.detach().contiguous())
        dA, dB = ftn.ftensordot_backward(ctx.A, ctx.B, DC, axes_a, axes_b, conv, gemm)
        return dA.data_view(), dB.data_view(), None, None, None, None, None, None, None


class _Transpose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, data, a, perm, out):
        T = ftn.ftranspose(a.handle(data), perm)
        out.append(T.legs())
        ctx.a, ctx.perm = a, perm
        return T.data_view()

    @staticmethod
    def backward(ctx, dt):
        a, perm = ctx.a, ctx.perm
        inv = [0] * len(perm)
        for i, p in enumerate(perm):
            inv[p] = i
        legs = [a.legs[p] for p in perm]
        D = ftn.Tensor.create(a.sym, legs, a.total, a.dtype, data=dt.detach().contiguous())
        return ftn.ftranspose(D, inv).data_view(), None, None, None


class _Compress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_data, b_data, a, b, la, lb, chi, cutoff, conv, out):
        A, B = a.handle(a_data), b.handle(b_data)
        A2, B2, _ = ftn.compress_bond(A, B, la, lb, chi, cutoff, conv)
        sa = (A2.legs(), A2.info()["total"])
        sb = (B2.legs(), B2.info()["total"])
        out.append((sa, sb))
        ctx.A, ctx.B = A, B
        ctx.args = (a.sym, la, lb, chi, cutoff, conv, sa, sb)
        return A2.data_view(), B2.data_view()

    @staticmethod
    def backward(ctx, dA2, dB2):
        sym, la, lb, chi, cutoff, conv, sa, sb = ctx.args
        DA = ftn.Tensor.create(sym, sa[0], sa[1], ftn.F64, data=dA2.detach().contiguous())
        DB = ftn.Tensor.create(sym, sb[0], sb[1], ftn.F64, data=dB2.detach().contiguous())
        da, db = ftn.compress_bond_backward(ctx.A, ctx.B, la, lb, chi, DA, DB, cutoff, conv)
        return da.data(), db.data(), None, None, None, None, None, None, None, None


def compress(a, b, la, lb, chi, cutoff=1e-12, conv=ftn.LOCAL):
    """Differentiable compress_bond of two FP64 DTensors (kept counts fixed).

    The backward pass is ``ftn_compress_bond_backward``, the derivative of
    the truncated SVD; it holds for losses that do not depend on the sign of
    each kept singular vector pair (e.g. any function of the product).
    """
    st = []
    da, db = _Compress.apply(a.data, b.data, a, b, int(la), int(lb), int(chi), float(cutoff), int(conv), st)
    (la_, ta), (lb_, tb) = st[0]
    return DTensor(a.sym, la_, ta, da), DTensor(b.sym, lb_, tb, db)


class _Fuse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, data, a, legs, conv, rev, out):
        A = a.handle(data)
        F = ftn.fuse(A, legs, conv, rev)
        sf = (F.legs(), F.info()["total"])
        out.append(sf)
        ctx.A = A
        ctx.args = (a.sym, a.dtype, legs, conv, rev, sf)
        return F.data()

    @staticmethod
    def backward(ctx, dF):
        sym, dtype, legs, conv, rev, sf = ctx.args
        D = ftn.Tensor.create(sym, sf[0], sf[1], dtype, data=dF.detach().contiguous())
        return ftn.fuse_backward(ctx.A, legs, D, conv, rev).data(), None, None, None, None, None


class _Dagger(torch.autograd.Function):
    @staticmethod
    def forward(ctx, data, a, out):
        A = a.handle(data)
        D = ftn.dagger(A)
        sd = (D.legs(), D.info()["total"])
        out.append(sd)
        ctx.args = (a.sym, a.dtype, sd)
        return D.data()

    @staticmethod
    def backward(ctx, dD):
        sym, dtype, sd = ctx.args
        G = ftn.Tensor.create(sym, sd[0], sd[1], dtype, data=dD.detach().contiguous())
        # the map is a permutation of entries without signs and an involution
        return ftn.dagger(G).data(), None, None


def dagger(a):
    """Differentiable Hermitian conjugate (legs reversed, duals flipped)."""
    st = []
    data = _Dagger.apply(a.data, a, st)
    return DTensor(a.sym, st[0][0], st[0][1], data)


def fuse(a, legs, conv=ftn.LOCAL, rev=0):
    """Differentiable fusion of the given legs of a DTensor (Sec. IV.A)."""
    st = []
    data = _Fuse.apply(a.data, a, [int(l) for l in legs], int(conv), int(rev), st)
    return DTensor(a.sym, st[0][0], st[0][1], data)


def dot(a, b, axes_a, axes_b, conv=ftn.LOCAL, gemm=ftn.GEMM_F64):
    """Differentiable ftensordot of two DTensors (output legs: free(a) ++ free(b))."""
    st = []
    data = _Dot.apply(a.data, b.data, a, b, [int(x) for x in axes_a], [int(x) for x in axes_b],
                      int(conv), int(gemm), st)
    legs, total = st[0]
    return DTensor(a.sym, legs, total, data)


def transpose(a, perm):
    """Differentiable ftranspose of a DTensor."""
    perm = [int(p) for p in perm]
    if sorted(perm) != list(range(a.ndim)):
        raise ValueError("not a permutation")
    st = []
    data = _Transpose.apply(a.data, a, perm, st)
    return DTensor(a.sym, st[0], a.total, data)


def add_dummy(a):
    """Prepend the size-1 odd dummy leg ('+', charge -s(T)); the data is unchanged."""
    if not a.parity:
        raise ValueError("add_dummy needs an odd tensor")
    q = _neg(a.sym, a.total)
    return DTensor(a.sym, [([q], [1], 0)] + a.legs, (0, 0), a.data)


def drop_leading_dummies(a, m):
    """Remove m leading size-1 dummy legs (block data unchanged)."""
    tot = a.total
    for (c, d, u) in a.legs[:m]:
        if len(c) != 1 or d != [1] or u != 0:
            raise ValueError("leg is not a dummy")
        tot = _sub(a.sym, tot, c[0])
    return DTensor(a.sym, a.legs[m:], tot, a.data)


def contract_exact(tensors, bonds, path, order=None, gemm=ftn.GEMM_F64):
    """Contract a network exactly in the local convention.

    ``tensors``: list of DTensor; ``bonds``: (t1, l1, t2, l2) with opposite
    duals; ``path``: SSA pairs; ``order``: global position of every tensor
    (sorts the dummy legs; default: list order). Returns ``(T, labels)``:
    the final DTensor (open legs only) and the (tensor, leg) of each leg.
    """
    n = len(tensors)
    T = dict(enumerate(tensors))
    lab = {t: [("o", t, l) for l in range(x.ndim)] for t, x in T.items()}
    for bi, (t1, l1, t2, l2) in enumerate(bonds):
        lab[t1][l1] = ("b", bi)
        lab[t2][l2] = ("b", bi)
    pos = list(range(n)) if order is None else [int(x) for x in order]
    for t in range(n):
        if T[t].parity:
            T[t] = add_dummy(T[t])
            lab[t] = [("d", t)] + lab[t]
    ssa = {i: i for i in range(n)}
    nid = n
    for (i, j) in path:
        x, y = ssa[i], ssa[j]
        pairs = [(k, lab[y].index(l)) for k, l in enumerate(lab[x]) if l[0] == "b" and l in lab[y]]
        pairs.sort(key=lambda p: lab[x][p[0]][1])
        lx, ly = [p[0] for p in pairs], [p[1] for p in pairs]
        T[nid] = dot(T[x], T[y], lx, ly, ftn.LOCAL, gemm)
        lab[nid] = [l for k, l in enumerate(lab[x]) if k not in lx] + [l for k, l in enumerate(lab[y]) if k not in ly]
        for t in (x, y):
            del T[t]
            del lab[t]
        ssa[len(ssa)] = nid
        nid += 1
    if len(T) != 1:
        raise ValueError("path does not contract the network to one tensor")
    (z, Z), = T.items()
    labs = lab[z]
    dpos = [k for k, l in enumerate(labs) if l[0] == "d"]
    m = len(dpos)
    if m:
        others = [k for k in range(Z.ndim) if k not in dpos]
        ds = sorted(dpos, key=lambda k: pos[labs[k][1]])
        Z = drop_leading_dummies(transpose(Z, ds + others), m)
        if (m * (m - 1) // 2) % 2:
            Z = DTensor(Z.sym, Z.legs, Z.total, -Z.data)
        labs = [labs[k] for k in others]
    return Z, [(l[1], l[2]) if l[0] == "o" else l for l in labs]


def network_value(tensors, bonds, path, order=None, gemm=ftn.GEMM_F64):
    """Value of a closed network as a 0-d torch tensor (differentiable)."""
    Z, labs = contract_exact(tensors, bonds, path, order, gemm)
    if Z.ndim:
        raise ValueError("network is not closed")
    return Z.data.sum()


class _NetState:
    """Host bookkeeping of a network contraction plus its live DTensors.

    ``T``: DTensors by id (consumed ids stay in the list); ``L``: labels of
    every leg (("o", tensor, leg) for open legs, ("b", bond) for bonds);
    ``D``: the dummy ranks each tensor carries; ``sgn``: the sign exponent of
    moving and merging them; ``e2``: binary exponent taken out so far.
    Steps replace list entries and never modify a DTensor or a label list in
    place, so a shallow copy of the lists is an independent state.
    """

    def __init__(self, tensors, bonds, pos):
        n = len(tensors)
        self.T = list(tensors)
        self.L = [[("o", t, l) for l in range(x.ndim)] for t, x in enumerate(tensors)]
        for bi, (t1, l1, t2, l2) in enumerate(bonds):
            self.L[t1][l1] = ("b", bi)
            self.L[t2][l2] = ("b", bi)
        odd = sorted([t for t in range(n) if self.T[t].parity], key=lambda t: pos[t])
        self.D = [[] for _ in range(n)]
        for r, t in enumerate(odd):
            self.D[t] = [r]
        self.sgn = 0
        self.alive = [True] * n
        self.ssa = list(range(n))
        self.next_bond = len(bonds)
        self.e2 = 0

    def copy(self):
        c = _NetState.__new__(_NetState)
        c.T, c.L, c.D, c.alive, c.ssa = list(self.T), list(self.L), list(self.D), list(self.alive), list(self.ssa)
        c.sgn, c.next_bond, c.e2 = self.sgn, self.next_bond, self.e2
        return c

    def shared(self, x, y):
        L = self.L
        pairs = [(L[x][k][1], k, L[y].index(l)) for k, l in enumerate(L[x]) if l[0] == "b" and l in L[y]]
        pairs.sort()
        return [p[1] for p in pairs], [p[2] for p in pairs]

    def step(self, i, j, chi, gemm):
        """One path step: dot, then fusion and compression of every bond of
        the new tensor, then the power-of-two rescaling."""
        import math
        T, L, D = self.T, self.L, self.D
        x, y = self.ssa[i], self.ssa[j]
        lx, ly = self.shared(x, y)
        Z = dot(T[x], T[y], lx, ly, ftn.LOCAL, gemm)
        e = (len(D[x]) & 1) & (len(D[y]) & 1)
        for a in D[x]:
            for b in D[y]:
                e ^= int(a > b)
        self.sgn ^= e
        D.append(sorted(D[x] + D[y]))
        L.append([l for k, l in enumerate(L[x]) if k not in lx] + [l for k, l in enumerate(L[y]) if k not in ly])
        T.append(Z)
        self.alive.append(True)
        self.alive[x] = self.alive[y] = False
        z = len(T) - 1
        self.ssa.append(z)
        if chi:
            nbs = [w for w in range(len(T)) if w != z and self.alive[w] and self.shared(z, w)[0]]
            for w in nbs:
                lz, lw = self.shared(z, w)
                if len(lz) > 1:
                    Tz, Tw = fuse(T[z], lz, ftn.LOCAL, 0), fuse(T[w], lw, ftn.LOCAL, 0)
                    nb = ("b", self.next_bond)
                    self.next_bond += 1
                    for t_, ls, X in ((z, lz, Tz), (w, lw, Tw)):
                        rest = [l for k, l in enumerate(L[t_]) if k not in ls]
                        p_ = sum(1 for k in range(len(L[t_])) if k not in ls and k < ls[0])
                        L[t_] = rest[:p_] + [nb] + rest[p_:]
                        T[t_] = X
                    lz, lw = self.shared(z, w)
                dim = sum(T[z].legs[lz[0]][1])
                if dim > chi and T[z].data.numel() and T[w].data.numel():
                    T[z], T[w] = compress(T[z], T[w], lz[0], lw[0], chi, 1e-12, ftn.LOCAL)
        m = float(T[z].data.detach().abs().max()) if T[z].data.numel() else 0.0
        if m > 0 and math.isfinite(m):
            ex = math.frexp(m)[1]
            T[z] = DTensor(T[z].sym, T[z].legs, T[z].total, T[z].data * (2.0 ** -ex))
            self.e2 += ex


class _Segment(torch.autograd.Function):
    """Recomputation checkpoint over consecutive path steps.

    The forward pass receives the outputs already computed without a graph
    and keeps only the segment's input data; the backward pass replays the
    segment from them with the graph recorded and back-propagates through
    it. The replay calls the same deterministic kernels on the same inputs,
    so it rebuilds the same block structures and values.
    """

    @staticmethod
    def forward(ctx, replay, outs, *ins):
        ctx.replay = replay
        ctx.save_for_backward(*ins)
        return tuple(o.detach() for o in outs)

    @staticmethod
    def backward(ctx, *gouts):
        ins = [x.detach().requires_grad_(True) for x in ctx.saved_tensors]
        with torch.enable_grad():
            outs = ctx.replay(ins)
        os_, gs_ = [], []
        for o, g in zip(outs, gouts):
            if g is not None and o.requires_grad:
                os_.append(o)
                gs_.append(g)
        if os_:
            torch.autograd.backward(os_, gs_)
        return (None, None) + tuple(x.grad for x in ins)


def _run_segment(st, steps, chi, gemm):
    """Advance ``st`` over ``steps`` (SSA pairs) under a recomputation
    checkpoint and return the new state."""
    with torch.no_grad():
        s1 = st.copy()
        for (i, j) in steps:
            s1.step(i, j, chi, gemm)
    n0 = len(st.T)
    ins = [t for t in range(n0) if st.alive[t] and (not s1.alive[t] or s1.T[t] is not st.T[t])]
    outs = [t for t in range(len(s1.T)) if s1.alive[t] and (t >= n0 or s1.T[t] is not st.T[t])]

    def replay(datas):
        s2 = st.copy()
        for t, d in zip(ins, datas):
            x = st.T[t]
            s2.T[t] = DTensor(x.sym, x.legs, x.total, d)
        for (i, j) in steps:
            s2.step(i, j, chi, gemm)
        return [s2.T[t].data for t in outs]

    datas = _Segment.apply(replay, [s1.T[t].data for t in outs], *[st.T[t].data for t in ins])
    for t, d in zip(outs, datas):
        x = s1.T[t]
        s1.T[t] = DTensor(x.sym, x.legs, x.total, d)
    return s1


def contract(tensors, bonds, path, chi=None, order=None, gemm=ftn.GEMM_F64, checkpoint=None):
    """Approximate (chi) or exact contraction, differentiable.

    The same steps as ``ftn_contract_network`` in the local convention, each
    a differentiable library call: pairwise ``dot`` over all shared bonds
    (paired in bond order), then for every neighbour (in creation order)
    the shared bonds fused into one and a bond larger than chi compressed
    (cutoff 1e-12, as the library's network driver), then a rescaling by a power of two. Odd tensors carry
    dummy ranks (by ``order``) whose moves and final sort are a sign.
    Returns ``(T, labels, exp2)``: the final DTensor scaled by 2^-exp2 and
    the (tensor, leg) of each open leg.

    ``checkpoint=s`` (s >= 1) runs the path in segments of s steps whose
    intermediates are not kept for the backward pass: only the tensors
    entering each segment (the environments at its boundary) are stored,
    and the backward pass recomputes one segment at a time. The gradient is
    the same; the cost is one more forward pass.
    """
    n = len(tensors)
    pos = list(range(n)) if order is None else [int(x) for x in order]
    st = _NetState(tensors, bonds, pos)
    path = [(int(i), int(j)) for (i, j) in path]
    if checkpoint is not None and int(checkpoint) >= 1 and torch.is_grad_enabled():
        s = int(checkpoint)
        for k0 in range(0, len(path), s):
            st = _run_segment(st, path[k0:k0 + s], chi, gemm)
    else:
        for (i, j) in path:
            st.step(i, j, chi, gemm)
    fin = [t for t in range(len(st.T)) if st.alive[t]]
    if len(fin) != 1:
        raise ValueError("path does not contract the network to one tensor")
    F = st.T[fin[0]]
    m = len(st.D[fin[0]])
    if ((m * (m - 1) // 2) & 1) ^ st.sgn:
        F = DTensor(F.sym, F.legs, F.total, -F.data)
    labs = [(l[1], l[2]) if l[0] == "o" else l for l in st.L[fin[0]]]
    return F, labs, st.e2


def norm_tensors(spec, kets, op=None, op_sites=None):
    """DTensors, bonds and global positions of <psi|psi> (or <psi|G|psi>).

    Tensor ids as in the library's norm networks: bra of site s is s (the
    dagger of the ket), ket of site s is n + s, the two-site operator 2n
    (legs out_u, out_v, in_v, in_u); positions follow Fig. 4(a).
    """
    from synth.workloads import norm_network_bonds, norm_network_positions
    n = spec.n_sites
    tensors = [dagger(k) for k in kets] + list(kets) + ([op] if op is not None else [])
    bonds = [(t1, l1, t2, l2) for (t1, l1, t2, l2, _) in
             norm_network_bonds(spec, op_sites if op is not None else None)]
    return tensors, bonds, norm_network_positions(n, op is not None)


def expectation_ratio(spec, kets, terms, paths, chi=None, gemm=ftn.GEMM_F64, checkpoint=None):
    """sum_t <psi|G_t|psi> / <psi|psi> as a 0-d torch tensor (differentiable).

    ``terms``: list of (G DTensor, (u, v)); ``paths``: {None: norm path,
    (u, v): path of that term}. Every network is contracted approximately
    with compression to chi (exact when chi is None), with recomputation
    checkpoints every ``checkpoint`` steps when given (see ``contract``).
    """
    t, b, p = norm_tensors(spec, kets)
    N, _, eN = contract(t, b, paths[None], chi, p, gemm, checkpoint)
    nval = N.data.sum()
    tot = 0.0
    for G, sites in terms:
        t, b, p = norm_tensors(spec, kets, G, sites)
        X, _, eX = contract(t, b, paths[tuple(sites)], chi, p, gemm, checkpoint)
        tot = tot + X.data.sum() * (2.0 ** (eX - eN))
    return tot / nval
