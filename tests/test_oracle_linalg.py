"""Pins of QR, truncated SVD and bond compression (CPU only).

* F(QR) reproduces the transposed tensor, Q is an isometry (Sec. II.A/B).
* Singular values equal numpy's SVD of the dense matrix of the transposed
  tensor (a +-1 change of row and column signs leaves them unchanged).
* Eckart-Young: the compressed pair reproduces the best rank-chi
  approximation of the dense bipartition matrix, with the discarded weight
  equal to the sum of the dropped s^2.
"""

import numpy as np
import pytest

from oracle import symmetry as S
from oracle.linalg import qr, svd, compress_bond
from oracle.ops import ftensordot, ftranspose
from tests.helpers import rand_leg, partner, rand_tensor


@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_qr_reconstructs_and_is_isometric(sym):
    rng = np.random.default_rng(20)
    for trial in range(5):
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(4)]
        T = rand_tensor(rng, sym, legs)
        rows = list(rng.permutation(4)[:2])
        cols = [i for i in range(4) if i not in rows]
        Q, R = qr(T, rows)
        back = ftensordot(Q, R, [Q.ndim - 1], [0], "local")
        ref = ftranspose(T, rows + cols)
        np.testing.assert_allclose(back.to_dense(), ref.to_dense(), atol=1e-12)
        # Q^T Q = 1 per block: contract Q with itself over the row legs
        Qd = Q.to_dense().reshape(-1, Q.legs[-1].size)
        G = Qd.T @ Qd
        np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-12)
        assert Q.total == T.total and R.total == S.zero(sym)


@pytest.mark.parametrize("sym", [S.Z2, S.U1U1])
def test_svd_values_match_dense(sym):
    rng = np.random.default_rng(21)
    for trial in range(5):
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(4)]
        T = rand_tensor(rng, sym, legs)
        rows = [0, 2]
        U, sv, V = svd(T, rows)
        got = np.sort(np.concatenate([v.numpy() for v in sv.values()]))[::-1]
        Td = ftranspose(T, [0, 2, 1, 3]).to_dense()
        M = Td.reshape(Td.shape[0] * Td.shape[1], -1)
        ref = np.linalg.svd(M, compute_uv=False)
        ref = ref[ref > 1e-12 * ref[0]]
        got = got[got > 1e-12 * got[0]]
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_compress_bond_eckart_young(conv, sym):
    rng = np.random.default_rng(22)
    for trial in range(6):
        bond = rand_leg(rng, sym, maxd=4)
        la = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        lb = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        pa = int(rng.integers(0, 3))
        pb = int(rng.integers(0, 3))
        A_legs = la[:pa] + [bond] + la[pa:]
        B_legs = lb[:pb] + [partner(bond)] + lb[pb:]
        A = rand_tensor(rng, sym, A_legs, total=S.zero(sym))
        B = rand_tensor(rng, sym, B_legs, total=S.zero(sym))
        C = ftensordot(A, B, [pa], [pb], conv)
        Cd = C.to_dense()
        M = Cd.reshape(Cd.shape[0] * Cd.shape[1], -1)
        s = np.linalg.svd(M, compute_uv=False)
        rank = int((s > 1e-12 * s[0]).sum())
        chi = max(1, rank - 2)
        A2, B2, info = compress_bond(A, B, pa, pb, chi, conv=conv)
        assert A2.legs[pa].size <= chi and A2.legs[pa].dual == A.legs[pa].dual
        C2 = ftensordot(A2, B2, [pa], [pb], conv)
        C2d = C2.to_dense()
        err2 = float(((Cd - C2d) ** 2).sum())
        ref_err2 = float((s[chi:] ** 2).sum())
        assert abs(err2 - ref_err2) <= 1e-10 * max(1.0, float((s ** 2).sum()))
        assert abs(info["discarded"] - ref_err2) <= 1e-10 * max(1.0, float((s ** 2).sum()))
        kept = np.sort(np.concatenate([v.numpy() for v in info["svals"].values()]))[::-1]
        np.testing.assert_allclose(kept, s[:chi], rtol=1e-10)
        # chi >= rank: exact
        A3, B3, _ = compress_bond(A, B, pa, pb, rank + 5, conv=conv)
        np.testing.assert_allclose(ftensordot(A3, B3, [pa], [pb], conv).to_dense(), Cd, atol=1e-10)


def test_select_top_exact_ties_across_charges():
    # the paper keeps the chi largest values over all blocks and is silent on
    # ties; the reading is: larger value first, then lower charge, then lower
    # index inside the sector; values not above cutoff * s_max are dropped
    from oracle.linalg import select_top
    sv = [(-1.0, (1,), 0), (-1.0, (0,), 0), (-0.5, (1,), 1), (-0.5, (0,), 1), (-0.25, (0,), 2)]
    assert select_top(sv, 1, 0.0) == {(0,): 1}
    assert select_top(sv, 2, 0.0) == {(0,): 1, (1,): 1}
    assert select_top(sv, 3, 0.0) == {(0,): 2, (1,): 1}
    assert select_top(sv, 4, 0.0) == {(0,): 2, (1,): 2}
    assert select_top(sv, None, 0.0) == {(0,): 3, (1,): 2}
    assert select_top(sv, None, 0.25) == {(0,): 2, (1,): 2}       # 0.25 is not above 0.25
    assert select_top(sv, None, 0.2499) == {(0,): 3, (1,): 2}
    # U(1)xU(1): charges compare lexicographically
    sv2 = [(-2.0, (0, 1), 0), (-2.0, (-1, 0), 0), (-2.0, (0, -1), 0), (-1.0, (-1, 0), 1)]
    assert select_top(sv2, 1, 0.0) == {(-1, 0): 1}
    assert select_top(sv2, 2, 0.0) == {(-1, 0): 1, (0, -1): 1}
    assert select_top(sv2, 3, 0.0) == {(-1, 0): 1, (0, -1): 1, (0, 1): 1}


def test_compress_bond_breaks_exact_ties_by_charge():
    # A~ = diag per sector, B~ = identity: the bond matrix of each Z2 sector
    # has singular values (3, 1) exactly, so the two sectors tie value by
    # value and the kept dims follow the tie-break alone
    from oracle.tensor import make_leg, FTensor
    import torch
    sym = S.Z2
    phys = make_leg(sym, [(0,), (1,)], [2, 2], 0)
    bond = make_leg(sym, [(0,), (1,)], [2, 2], 1)
    A = FTensor.zeros(sym, [phys, bond], (0,))
    B = FTensor.zeros(sym, [partner(bond), partner(phys)], (0,))
    for q in (0, 1):
        A.blocks[(q, q)] = torch.diag(torch.tensor([3.0, 1.0], dtype=torch.float64))
        B.blocks[(q, q)] = torch.eye(2, dtype=torch.float64)
    for chi, dims in ((1, ((0,),)), (2, ((0,), (1,))), (3, ((0,), (1,)))):
        A2, B2, info = compress_bond(A, B, 1, 0, chi)
        assert A2.legs[1].charges == dims
        kept = {q: len(v) for q, v in info["svals"].items()}
        want = {1: {(0,): 1}, 2: {(0,): 1, (1,): 1}, 3: {(0,): 2, (1,): 1}}[chi]
        assert kept == want
        assert abs(info["discarded"] - {1: 11.0, 2: 2.0, 3: 1.0}[chi]) <= 1e-12
