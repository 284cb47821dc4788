"""Pins of the oracle's elementary operations (CPU only).

Each test checks the oracle against something other than its own code: a
closed-form count, the paper's printed worked example (Eq. standardcontract)
and Z2 identity (Sec. II.B, swap rule), the adjacent-swap rule (Eq.
transposition), group-action algebra, and the bosonic limit (Sec. II.C:
all-even legs behave as ordinary arrays).
"""

import itertools

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from oracle.tensor import FTensor, make_leg, enumerate_keys
from oracle.ops import (ftranspose, ftensordot, flip_dual, koszul, dagger,
                        tensordot_bosonic, add_dummy, leg_parity_sign)
from oracle.dense import leg_parity_vector
from tests.helpers import rand_leg, partner, rand_tensor


# --- block enumeration (Eq. symmetryrule) ---------------------------------

@pytest.mark.parametrize("n,e,o", [(1, 1, 1), (3, 2, 1), (4, 2, 2), (5, 1, 3)])
@pytest.mark.parametrize("tot", [0, 1])
def test_z2_allowed_count_closed_form(n, e, o, tot):
    # number of entries with even (odd) total parity: ((e+o)^n +- (e-o)^n)/2
    legs = [make_leg(S.Z2, [(0,), (1,)], [e, o], i % 2) for i in range(n)]
    T = FTensor.zeros(S.Z2, legs, (tot,))
    expect = ((e + o) ** n + (1 - 2 * tot) * (e - o) ** n) // 2
    assert T.nnz() == expect


def test_u1_allowed_count_generating_function():
    # U(1): count = coefficient of x^s in prod_i P_i(x^{sigma_i}) (polymul)
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(1, 5))
        legs, polys = [], []
        for i in range(n):
            ch = sorted(set(int(x) for x in rng.integers(-2, 3, size=3)))
            dims = [int(x) for x in rng.integers(1, 3, size=len(ch))]
            dual = int(rng.integers(0, 2))
            legs.append(make_leg(S.U1, [(c,) for c in ch], dims, dual))
            # polynomial over exponent range [-2, 2] shifted by 2
            p = np.zeros(5)
            for c, d in zip(ch, dims):
                p[(-c if dual else c) + 2] += d
            polys.append(p)
        tot = int(rng.integers(-2, 3))
        prod = np.array([1.0])
        for p in polys:
            prod = np.convolve(prod, p)
        # exponent offset is 2*n
        idx = tot + 2 * n
        expect = int(round(prod[idx])) if 0 <= idx < len(prod) else 0
        T = FTensor.zeros(S.U1, legs, (tot,))
        assert T.nnz() == expect


def test_keys_are_lexicographic_and_complete():
    rng = np.random.default_rng(2)
    legs = [rand_leg(rng, S.U1U1) for _ in range(3)]
    keys = enumerate_keys(S.U1U1, legs, (0, 0))
    assert keys == sorted(keys)
    dense_allowed = 0
    for idx in itertools.product(*[range(l.nsect) for l in legs]):
        q = [0, 0]
        for l, i in zip(legs, idx):
            s = -1 if l.dual else 1
            q[0] += s * l.charges[i][0]
            q[1] += s * l.charges[i][1]
        dense_allowed += (tuple(q) == (0, 0))
    assert len(keys) == dense_allowed


# --- transposition (Eq. transposition) -----------------------------------

@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_adjacent_swap_sign(sym):
    rng = np.random.default_rng(3)
    for trial in range(10):
        n = int(rng.integers(2, 5))
        legs = [rand_leg(rng, sym) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        i = int(rng.integers(0, n - 1))
        perm = list(range(n))
        perm[i], perm[i + 1] = perm[i + 1], perm[i]
        Tt = ftranspose(T, perm)
        D = T.to_dense()
        pi = leg_parity_vector(sym, legs[i])
        pj = leg_parity_vector(sym, legs[i + 1])
        shp = [1] * n
        shp[i] = len(pi)
        sgn_i = pi.reshape(shp)
        shp = [1] * n
        shp[i + 1] = len(pj)
        sgn_j = pj.reshape(shp)
        expect = np.transpose(D * (-1.0) ** (sgn_i * sgn_j), perm)
        np.testing.assert_array_equal(Tt.to_dense(), expect)


def test_transpose_group_action():
    rng = np.random.default_rng(4)
    for trial in range(20):
        n = int(rng.integers(2, 6))
        legs = [rand_leg(rng, S.Z2) for _ in range(n)]
        T = rand_tensor(rng, S.Z2, legs)
        p1 = list(rng.permutation(n))
        p2 = list(rng.permutation(n))
        a = ftranspose(ftranspose(T, p1), p2)
        comp = [p1[p2[t]] for t in range(n)]
        b = ftranspose(T, comp)
        np.testing.assert_array_equal(a.to_dense(), b.to_dense())
        inv = [0] * n
        for t, p in enumerate(p1):
            inv[p] = t
        np.testing.assert_array_equal(ftranspose(ftranspose(T, p1), inv).to_dense(), T.to_dense())


def test_koszul_cycle_closed_form():
    # moving one odd leg past m odd legs: sign (-1)^m
    for m in range(6):
        par = [1] * (m + 1)
        perm = list(range(1, m + 1)) + [0]
        assert koszul(par, perm) == m % 2


# --- contraction: worked example and bosonic limit -------------------------

def _dense_parity_grid(sym, legs):
    vecs = [leg_parity_vector(sym, l) for l in legs]
    return np.meshgrid(*vecs, indexing="ij")


@pytest.mark.parametrize("sym", [S.Z2, S.U1])
def test_worked_example_standardcontract(sym):
    # C_{ijlmnr} = sum_k (-1)^{p_k (p_l + p_m + p_n)} A_{ijkl} B_{mnkr}
    rng = np.random.default_rng(5)
    for trial in range(6):
        li, lj, lk, ll = [rand_leg(rng, sym) for _ in range(4)]
        lm, ln, lr = [rand_leg(rng, sym) for _ in range(3)]
        A = rand_tensor(rng, sym, [li, lj, lk, ll])
        B = rand_tensor(rng, sym, [lm, ln, partner(lk), lr])
        C = ftensordot(A, B, [2], [2], conv="global")
        Ad, Bd = A.to_dense(), B.to_dense()
        pk = leg_parity_vector(sym, lk)
        pl = leg_parity_vector(sym, ll)
        pm = leg_parity_vector(sym, lm)
        pn = leg_parity_vector(sym, ln)
        sgn = (-1.0) ** (pk[:, None, None, None] *
                         (pl[None, :, None, None] + pm[None, None, :, None] + pn[None, None, None, :]))
        expect = np.einsum("ijkl,klmn,mnkr->ijlmnr", Ad, sgn, Bd)
        np.testing.assert_allclose(C.to_dense(), expect, rtol=0, atol=1e-13)


def test_swap_rule_z2_identity_exhaustive():
    # (p_m+p_r)(p_k+p_s) + (p_r+p_k)p_n + (p_s+p_m)p_n = p_A p_B + p_n (mod 2)
    for pm, pn, pr, pk, ps in itertools.product((0, 1), repeat=5):
        pa = (pm + pn + pr) % 2
        pb = (pk + pn + ps) % 2
        lhs = ((pm + pr) * (pk + ps) + (pr + pk) * pn + (ps + pm) * pn) % 2
        assert lhs == (pa * pb + pn) % 2


@pytest.mark.parametrize("pa,pb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_swap_rule(pa, pb):
    # F(AB) = F(B g A) with g_n = (-1)^{p_n} (-1)^{p_A p_B}, Eq. (fermiswap):
    # T_{mrks} = sum^F_n A_{mnr} B_{kns}; T~_{ksmr} = sum^F_n B~_{kns} A~_{mnr}
    # equals (-1)^{(p_m+p_r)(p_k+p_s)} T_{mrks} (Eq. swapdefn).
    rng = np.random.default_rng(6)
    sym = S.Z2
    for trial in range(5):
        lm, ln, lr, lk, ls = [rand_leg(rng, sym) for _ in range(5)]
        A = rand_tensor(rng, sym, [lm, ln, lr], total=(pa,))
        B = rand_tensor(rng, sym, [lk, partner(ln), ls], total=(pb,))
        T = ftensordot(A, B, [1], [1], conv="global")            # legs m r k s
        # B~ = (-1)^{p_n} (-1)^{pA pB} B on leg n
        Bt = leg_parity_sign(B, 1)
        if pa * pb:
            Bt = Bt.scaled(-1.0)
        Tt = ftensordot(Bt, A, [1], [1], conv="global")          # legs k s m r
        back = ftranspose(Tt, [2, 3, 0, 1])                       # Koszul to m r k s
        np.testing.assert_allclose(back.to_dense(), T.to_dense(), atol=1e-13)


def test_bosonic_limit_all_even():
    # all-even legs: fermionic ops reduce to numpy transpose / tensordot
    rng = np.random.default_rng(7)
    legs = [make_leg(S.Z2, [(0,)], [3], d) for d in (0, 1, 0, 1)]
    A = rand_tensor(rng, S.Z2, legs, total=(0,))
    perm = [2, 0, 3, 1]
    np.testing.assert_array_equal(ftranspose(A, perm).to_dense(), np.transpose(A.to_dense(), perm))
    B = rand_tensor(rng, S.Z2, [make_leg(S.Z2, [(0,)], [3], 1 - legs[1].dual),
                                make_leg(S.Z2, [(0,)], [3], 0)], total=(0,))
    for conv in ("local", "global"):
        C = ftensordot(A, B, [1], [0], conv=conv)
        np.testing.assert_allclose(C.to_dense(), np.tensordot(A.to_dense(), B.to_dense(), ([1], [0])), atol=1e-13)


def test_local_convention_arrow_rule():
    # local: head ('-') on the left is sign-free; '+' on the left costs (-1)^p
    rng = np.random.default_rng(8)
    sym = S.Z2
    lb = make_leg(sym, [(0,), (1,)], [2, 2], 1)
    A = rand_tensor(rng, sym, [rand_leg(rng, sym), lb], total=(0,))
    B = rand_tensor(rng, sym, [partner(lb), rand_leg(rng, sym)], total=(0,))
    np.testing.assert_array_equal(ftensordot(A, B, [1], [0], "local").to_dense(),
                                  ftensordot(A, B, [1], [0], "global").to_dense())
    A2 = flip_dual(A, 1)
    B2 = flip_dual(B, 0)
    # reversing the bond (one g) keeps the local value
    np.testing.assert_allclose(ftensordot(A2, B2, [1], [0], "local").to_dense(),
                               ftensordot(A, B, [1], [0], "local").to_dense(), atol=1e-13)


@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_local_order_independence_even(sym):
    # for even tensors F_local(BA) is the fermionic transpose of F_local(AB)
    rng = np.random.default_rng(9)
    for trial in range(8):
        la = [rand_leg(rng, sym) for _ in range(3)]
        lb = [rand_leg(rng, sym) for _ in range(2)]
        k = int(rng.integers(1, 3))
        bond = [rand_leg(rng, sym) for _ in range(k)]
        A_legs = la + bond
        B_legs = [partner(b) for b in bond] + lb
        pa = list(rng.permutation(len(A_legs)))
        pb = list(rng.permutation(len(B_legs)))
        A = rand_tensor(rng, sym, [A_legs[p] for p in pa], total=S.zero(sym))
        B = rand_tensor(rng, sym, [B_legs[p] for p in pb], total=S.zero(sym))
        ax_a = [pa.index(3 + t) for t in range(k)]
        ax_b = [pb.index(t) for t in range(k)]
        AB = ftensordot(A, B, ax_a, ax_b, "local")
        BA = ftensordot(B, A, ax_b, ax_a, "local")
        na = A.ndim - k
        nb = B.ndim - k
        perm = list(range(nb, nb + na)) + list(range(nb))
        np.testing.assert_allclose(ftranspose(BA, perm).to_dense(), AB.to_dense(), atol=1e-12)


def test_parity_and_charge_conservation():
    rng = np.random.default_rng(10)
    for sym in (S.Z2, S.U1, S.U1U1):
        for trial in range(5):
            la = [rand_leg(rng, sym) for _ in range(3)]
            bond = rand_leg(rng, sym)
            A = rand_tensor(rng, sym, la + [bond])
            B = rand_tensor(rng, sym, [partner(bond), rand_leg(rng, sym)])
            C = ftensordot(A, B, [3], [0])
            assert C.total == S.add(sym, A.total, B.total)
            assert C.parity == (A.parity + B.parity) % 2
            # every stored block obeys the rule
            for key in C.blocks:
                q = S.zero(sym)
                for l, i in zip(C.legs, key):
                    q = S.add(sym, q, S.signed(sym, l.dual, l.charges[i]))
                assert q == C.total


def test_dagger_and_dummy():
    rng = np.random.default_rng(11)
    legs = [rand_leg(rng, S.Z2) for _ in range(3)]
    T = rand_tensor(rng, S.Z2, legs, total=(1,))
    Td = dagger(T)
    np.testing.assert_array_equal(Td.to_dense(), np.transpose(T.to_dense(), [2, 1, 0]))
    assert [l.dual for l in Td.legs] == [1 - l.dual for l in reversed(T.legs)]
    D = add_dummy(T)
    assert D.parity == 0 and D.ndim == 4 and D.legs[0].dims == (1,)
    np.testing.assert_array_equal(D.to_dense()[0], T.to_dense())


def test_scalar_tensors():
    # a tensor with no legs holds one entry iff its total charge is neutral
    T = FTensor.from_dense(S.Z2, [], (0,), np.array(2.5))
    assert T.keys() == [()] and float(T.block(())) == 2.5
    assert FTensor.from_dense(S.Z2, [], (1,), np.array(2.5)).keys() == []
    assert ftranspose(T, []).to_dense() == 2.5
