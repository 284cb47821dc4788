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
