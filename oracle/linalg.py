"""QR, truncated SVD and bond compression of fermionic tensors.

Sec. II.A: a symmetric tensor is decomposed as a matrix after grouping its
legs into rows and columns; for QR the factor Q keeps s(A) and R is neutral,
for SVD U keeps s(A), and truncation keeps the chi largest singular values
taken over all symmetry blocks together. Sec. II.B: for fermionic tensors
the grouping is preceded by the fermionic transposition to rows ++ columns.

The matrices are the per-charge blocks of the grouped tensor: for a column
charge c (the sigma-weighted sum of the column legs' charges) the rows are
all row-key combinations whose charge complements c, stacked in
lexicographic key order. Decompositions call ``torch.linalg`` in FP64.

Truncation tie-break (the paper is silent): sort by (-s, charge of the
sector, index inside the sector), keep the first chi, drop values not above
``cutoff * s_max``, drop sectors left empty.
"""

import numpy as np
import torch

from . import symmetry as S
from .ops import ftranspose, ftensordot
from .tensor import FTensor, Leg


def _row_keys(sym, legs):
    import itertools
    out = []
    for key in itertools.product(*[range(l.nsect) for l in legs]):
        q = S.zero(sym)
        d = 1
        for l, i in zip(legs, key):
            q = S.add(sym, q, S.signed(sym, l.dual, l.charges[i]))
            d *= l.dims[i]
        out.append((key, q, d))
    return out


def group_matrices(T, nrow):
    """Matrices of T (already ordered rows ++ cols) per column charge.

    Returns {c: (M, row_list, col_list)} where row_list/col_list hold
    (key, dim) pairs in stacking order.
    """
    sym = T.sym
    rows = _row_keys(sym, T.legs[:nrow])
    cols = _row_keys(sym, T.legs[nrow:])
    out = {}
    col_by_c = {}
    for key, q, d in cols:
        col_by_c.setdefault(q, []).append((key, d))
    for c, clist in sorted(col_by_c.items()):
        need = S.add(sym, T.total, S.neg(sym, c))
        rlist = [(k, d) for (k, q, d) in rows if q == need]
        m = sum(d for _, d in rlist)
        n = sum(d for _, d in clist)
        M = torch.zeros((m, n), dtype=torch.float64)
        r0 = 0
        for rk, rd in rlist:
            c0 = 0
            for ck, cd in clist:
                blk = T.block(tuple(rk) + tuple(ck))
                M[r0:r0 + rd, c0:c0 + cd] = blk.reshape(rd, cd)
                c0 += cd
            r0 += rd
        out[c] = (M, rlist, clist)
    return out


def qr(T, row_legs):
    """Q R = T~ with T~ = T transposed to rows ++ cols (Sec. II.A, II.B).

    The new leg is the last leg of Q ('-') and the first of R ('+'); its
    sector label is -c for column charge c, so Q keeps s(T) and R is neutral
    and F(QR) = T~ carries no extra sign.
    """
    return _decompose(T, row_legs, "qr")


def svd(T, row_legs, chi=None, cutoff=0.0):
    """U, S, V with U keeping s(T); truncation to the global top chi."""
    return _decompose(T, row_legs, "svd", chi=chi, cutoff=cutoff)


def _decompose(T, row_legs, kind, chi=None, cutoff=0.0):
    sym = T.sym
    row_legs = [int(i) for i in row_legs]
    col_legs = [i for i in range(T.ndim) if i not in row_legs]
    Tt = ftranspose(T, row_legs + col_legs)
    nrow = len(row_legs)
    mats = group_matrices(Tt, nrow)
    facs = {}
    svals = []
    for c, (M, rl, cl) in mats.items():
        if M.shape[0] == 0 or M.shape[1] == 0:
            continue
        if kind == "qr":
            Q, R = torch.linalg.qr(M, mode="reduced")
            facs[c] = (Q, R, rl, cl)
        else:
            U, s, Vh = torch.linalg.svd(M, full_matrices=False)
            facs[c] = (U, s, Vh, rl, cl)
            for i, v in enumerate(s.tolist()):
                svals.append((-v, c, i))
    keep = None
    if kind == "svd":
        keep = select_top(svals, chi, cutoff)
    labels = sorted(S.neg(sym, c) for c in facs)
    lab_of = {c: S.neg(sym, c) for c in facs}
    dims = {}
    for c in facs:
        if kind == "qr":
            dims[c] = facs[c][1].shape[0]
        else:
            dims[c] = keep.get(c, 0)
    chs = [q for q in labels if dims[S.neg(sym, q)] > 0]
    newdims = [dims[S.neg(sym, q)] for q in chs]
    leg_l = Leg(tuple(chs), tuple(newdims), 1)
    leg_r = Leg(tuple(chs), tuple(newdims), 0)
    left = FTensor.zeros(sym, list(Tt.legs[:nrow]) + [leg_l], Tt.total)
    right = FTensor.zeros(sym, [leg_r] + list(Tt.legs[nrow:]), S.zero(sym))
    smap = {}
    for c, f in facs.items():
        k = dims[c]
        if k == 0:
            continue
        if kind == "qr":
            L, Rm, rl, cl = f
            Rm = Rm[:k]
            L = L[:, :k]
        else:
            U, s, Vh, rl, cl = f
            L = U[:, :k]
            Rm = Vh[:k]
            smap[lab_of[c]] = s[:k]
        li = leg_l.charges.index(lab_of[c])
        r0 = 0
        for rk, rd in rl:
            key = tuple(rk) + (li,)
            shp = left.shape_of(key)
            left.blocks[key] = L[r0:r0 + rd].reshape(shp).clone()
            r0 += rd
        c0 = 0
        for ck, cd in cl:
            key = (li,) + tuple(ck)
            shp = right.shape_of(key)
            right.blocks[key] = Rm[:, c0:c0 + cd].reshape(shp).clone()
            c0 += cd
    if kind == "qr":
        return left, right
    return left, smap, right


def select_top(svals, chi, cutoff):
    """Global top-chi over all blocks; returns {charge: count kept}."""
    if not svals:
        return {}
    smax = -min(v for v, _, _ in svals)
    order = sorted(svals)
    keep = {}
    n = 0
    for negv, c, i in order:
        if chi is not None and n >= chi:
            break
        if -negv <= cutoff * smax:
            break
        keep[c] = keep.get(c, 0) + 1
        n += 1
    return keep


def near_tie(svals, chi, rel=1e3 * np.finfo(np.float64).eps):
    """True if the chi-th and (chi+1)-th largest values are within ``rel``."""
    vs = sorted((-v for v, _, _ in svals), reverse=True)
    if chi is None or len(vs) <= chi or chi == 0:
        return False
    a, b = vs[chi - 1], vs[chi]
    return abs(a - b) <= rel * max(abs(a), 1e-300)


class _TruncatedSVD(torch.autograd.Function):
    """(A', B') = (U_k S_k^1/2, S_k^1/2 V_k^T) for C = MA MB = U S V^T.

    Backward: the derivative of the leading k singular triplets (Sec. II.A
    truncated SVD). With Gu = dA' S^1/2, Gv = dB'^T S^1/2, a = U^T Gu,
    b = V^T Gv over the r nonzero singular values (> 1e-12 s_max),
        dC = U Y V^T + (I - U U^T) Gu S_k^-1 V_k^T + U_k S_k^-1 Gv^T (I - V V^T),
        Y[x, y] = [y < k] (a[x, y] s_y + b[x, y] s_x) / (s_y^2 - s_x^2)
                + [x < k] (a[y, x] s_y + b[y, x] s_x) / (s_x^2 - s_y^2)   (x != y)
        Y[x, x] = [x < k] (a[x, x] + b[x, x]) / (2 s_x),
    then dMA = dC MB^T, dMB = MA^T dC. Pairs of singular values closer than
    1e-13 s_max^2 are treated as degenerate: a loss that is a function of the
    compressed product does not depend on the rotation inside such a pair,
    and its coupling term is zero.
    """

    @staticmethod
    def forward(ctx, MA, MB, k):
        C = MA @ MB
        U, s, Vh = torch.linalg.svd(C, full_matrices=False)
        sq = torch.sqrt(s[:k])
        ctx.save_for_backward(MA, MB, U, s, Vh)
        ctx.k = k
        return U[:, :k] * sq[None, :], sq[:, None] * Vh[:k]

    @staticmethod
    def backward(ctx, dA, dB):
        MA, MB, U, s, Vh = ctx.saved_tensors
        k = ctx.k
        r = int((s > 1e-12 * s[0]).sum()) if s.numel() and s[0] > 0 else 0
        U, V, s = U[:, :r], Vh[:r].T, s[:r]
        sk = s[:k]
        Gu = dA * torch.sqrt(sk)[None, :]
        Gv = dB.T * torch.sqrt(sk)[None, :]
        a = U.T @ Gu
        b = V.T @ Gv
        tie = 1e-13 * float(s[0]) ** 2 if r else 0.0
        den = s[None, :] ** 2 - s[:, None] ** 2          # den[x, y] = s_y^2 - s_x^2
        ok = den.abs() > tie                               # excludes x == y
        safe = torch.where(ok, den, torch.ones_like(den))
        Y = torch.zeros((r, r), dtype=torch.float64)
        t1 = (a * s[None, :k] + b * s[:, None]) / safe[:, :k]          # y < k
        Y[:, :k] += torch.where(ok[:, :k], t1, torch.zeros_like(t1))
        t2 = (a.T * s[None, :] + b.T * s[:k, None]) / safe[:k, :]      # x < k
        Y[:k, :] -= torch.where(ok[:k, :], t2, torch.zeros_like(t2))
        idx = torch.arange(k)
        Y[idx, idx] = (a[idx, idx] + b[idx, idx]) / (2 * sk)
        dC = U @ Y @ V.T
        dC = dC + (Gu - U @ a) @ (V[:, :k] / sk[None, :]).T
        dC = dC + (U[:, :k] / sk[None, :]) @ (Gv - V @ b).T
        return dC @ MB.T, MA.T @ dC, None



def compress_bond(A, B, la, lb, chi, conv="local", cutoff=1e-12):
    """Truncate the single bond (A leg ``la``, B leg ``lb``) to at most chi.

    Steps (the paper names the operation, Sec. III, but not its algorithm):
    (1) A~ = A with ``la`` moved last, B~ = B with ``lb`` moved first
    (fermionic transpositions); in the local convention the bond parity of
    Eq. (fermionictn2) is folded into B~ when A's end is '+'. (2) Per bond
    charge q: A~_q = Q_A R_A, B~_q = L_B Q_B, X = R_A L_B = U S V^T.
    (3) Keep the global top chi singular values. (4) A' = Q_A U sqrt(S),
    B' = sqrt(S) V^T Q_B; the bond parity is removed from B' again and both
    tensors are transposed back so the bond keeps its leg position, dual and
    charges. Then F(A'B') is the best rank-chi approximation of F(AB) across
    the bond.

    Returns ``(A', B', info)`` with info keys ``discarded`` (sum of dropped
    s^2), ``svals`` ({charge: kept values}), ``all_svals``, ``near_tie``.
    """
    sym = A.sym
    LA, LB = A.legs[la], B.legs[lb]
    if LA.dual == LB.dual:
        raise ValueError("bond legs must have opposite duals")
    rest_a = [i for i in range(A.ndim) if i != la]
    rest_b = [i for i in range(B.ndim) if i != lb]
    At = ftranspose(A, rest_a + [la])
    Bt = ftranspose(B, [lb] + rest_b)
    fold = conv == "local" and LA.dual == 0
    if fold:
        Bt = _bond_sign(Bt, 0)
    # B~ per bond sector q: rows = the sector, columns = B's blocks with it
    bmats = {}
    for qi, q in enumerate(Bt.legs[0].charges):
        cl = []
        for key in Bt.keys():
            if key[0] == qi:
                cl.append(key)
        d = Bt.legs[0].dims[qi]
        n = sum(int(np.prod(Bt.shape_of(k)[1:])) for k in cl)
        M = torch.zeros((d, n), dtype=torch.float64)
        c0 = 0
        for key in cl:
            shp = Bt.shape_of(key)
            w = int(np.prod(shp[1:]))
            M[:, c0:c0 + w] = Bt.block(key).reshape(d, w)
            c0 += w
        bmats[q] = (M, cl)
    # A~ per bond sector q: columns = the sector, rows = A's blocks with it
    amats = {}
    for qi, q in enumerate(At.legs[-1].charges):
        rl = [key for key in At.keys() if key[-1] == qi]
        d = At.legs[-1].dims[qi]
        m = sum(int(np.prod(At.shape_of(k)[:-1])) for k in rl)
        M = torch.zeros((m, d), dtype=torch.float64)
        r0 = 0
        for key in rl:
            shp = At.shape_of(key)
            h = int(np.prod(shp[:-1]))
            M[r0:r0 + h] = At.block(key).reshape(h, d)
            r0 += h
        amats[q] = (M, rl)
    facs = {}
    svals = []
    for q in At.legs[-1].charges:
        if q not in bmats:
            continue
        MA, rl = amats[q]
        MB, cl = bmats[q]
        if MA.shape[0] == 0 or MB.shape[1] == 0:
            continue
        if MA.requires_grad or MB.requires_grad:
            # derivatives go through the SVD of the bond matrix itself, with
            # the textbook adjoint (_TruncatedSVD): reverse mode through the QR
            # of a rank-deficient factor divides by its zero pivots, and
            # through torch's SVD by differences of equal zero singular values
            s = torch.linalg.svdvals((MA @ MB).detach())
            facs[q] = (None, (MA, MB), s, None, None, rl, cl)
        else:
            QA, RA = torch.linalg.qr(MA, mode="reduced")
            QBt, RBt = torch.linalg.qr(MB.T, mode="reduced")
            LBm = RBt.T
            QB = QBt.T
            X = RA @ LBm
            U, s, Vh = torch.linalg.svd(X, full_matrices=False)
            facs[q] = (QA, U, s, Vh, QB, rl, cl)
        for i, v in enumerate(s.tolist()):
            svals.append((-v, q, i))
    keep = select_top(svals, chi, cutoff)
    kept_total = sum(v * v for v in (-x for x, _, _ in svals))
    chs = [q for q in At.legs[-1].charges if keep.get(q, 0) > 0]
    dims = [keep[q] for q in chs]
    new_a = Leg(tuple(chs), tuple(dims), LA.dual)
    new_b = Leg(tuple(chs), tuple(dims), LB.dual)
    Ap = FTensor.zeros(sym, list(At.legs[:-1]) + [new_a], A.total)
    Bp = FTensor.zeros(sym, [new_b] + list(Bt.legs[1:]), B.total)
    discarded = 0.0
    sv_out = {}
    for q, (QA, U, s, Vh, QB, rl, cl) in facs.items():
        k = keep.get(q, 0)
        discarded += float((s[k:] ** 2).sum().detach())
        if k == 0:
            continue
        if QA is None:  # differentiable route: U holds the factors (MA, MB)
            LA_, RB_ = _TruncatedSVD.apply(U[0], U[1], k)
        else:
            sq = torch.sqrt(s[:k])
            LA_ = (QA @ U[:, :k]) * sq[None, :]
            RB_ = (sq[:, None] * Vh[:k]) @ QB
        sv_out[q] = s[:k]
        qi = chs.index(q)
        r0 = 0
        for key in rl:
            nk = tuple(key[:-1]) + (qi,)
            shp = Ap.shape_of(nk)
            h = int(np.prod(shp[:-1]))
            Ap.blocks[nk] = LA_[r0:r0 + h].reshape(shp).clone()
            r0 += h
        c0 = 0
        for key in cl:
            nk = (qi,) + tuple(key[1:])
            shp = Bp.shape_of(nk)
            w = int(np.prod(shp[1:]))
            Bp.blocks[nk] = RB_[:, c0:c0 + w].reshape(shp).clone()
            c0 += w
    if fold:
        Bp = _bond_sign(Bp, 0)
    inv_a = [0] * A.ndim
    for t, p in enumerate(rest_a + [la]):
        inv_a[p] = t
    inv_b = [0] * B.ndim
    for t, p in enumerate([lb] + rest_b):
        inv_b[p] = t
    Ap = ftranspose(Ap, inv_a)
    Bp = ftranspose(Bp, inv_b)
    info = dict(discarded=discarded, svals=sv_out, all_svals=svals,
                near_tie=near_tie(svals, chi), total=kept_total)
    return Ap, Bp, info


def _bond_sign(T, leg):
    out = FTensor(T.sym, T.legs, T.total)
    for key in T.keys():
        p = S.parity(T.sym, T.legs[leg].charges[key[leg]])
        out.blocks[key] = -T.block(key) if p else T.block(key).clone()
    return out
