"""Pins of network contraction in the oracle (CPU only).

* Koszul brute force (global convention, Sec. II.D) on random tiny
  networks with random duals, leg orders, odd tensors and open legs.
* Swap-gate bosonisation (the hand-inserted swap tensors of Sec. I).
* Contraction-order invariance (Sec. III) and the local convention
  (Sec. II.E) against the global one after the DAG translation.
* Fusion of parallel bonds (Sec. IV.A).
"""

import numpy as np
import pytest

from oracle import symmetry as S
from oracle import dense
from oracle.network import Network, contract_network, to_local
from oracle.ops import fuse, ftensordot, ftranspose
from tests.helpers import random_network, random_ssa_path, rand_leg, partner, rand_tensor


def _value_with_open(net, path):
    T, labs, e, _ = contract_network(net, path)
    return T, labs, e


def _to_flat_order(T, labs, order, tensors):
    """Transpose the result's open legs into flat (position) order."""
    flat = [("o", t, l) for t in order for l in range(tensors[t].ndim)]
    rank = {lab: k for k, lab in enumerate(flat)}
    perm = sorted(range(T.ndim), key=lambda k: rank[labs[k]])
    return ftranspose(T, perm)


@pytest.mark.parametrize("sym", [S.Z2, S.U1])
@pytest.mark.parametrize("seed", range(6))
def test_global_pairwise_equals_koszul_bruteforce(sym, seed):
    rng = np.random.default_rng(100 + seed)
    nt = int(rng.integers(2, 6))
    tensors, bonds = random_network(rng, sym, nt, nt + int(rng.integers(0, 2)),
                                    n_open=int(rng.integers(0, 3)), odd_frac=0.4)
    pos = list(rng.permutation(nt))
    order = sorted(range(nt), key=lambda t: pos[t])
    ref = dense.koszul_value(tensors, bonds, order)
    net = Network(tensors, bonds, conv="global", positions=pos)
    for trial in range(3):
        path = random_ssa_path(rng, tensors, bonds)
        T, labs, e = _value_with_open(net, path)
        T = _to_flat_order(T, labs, order, tensors)
        np.testing.assert_allclose(T.to_dense() * 2.0 ** e, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_swap_gates_equal_koszul_closed(seed):
    rng = np.random.default_rng(200 + seed)
    nt = int(rng.integers(2, 6))
    tensors, bonds = random_network(rng, S.Z2, nt, nt + 1, n_open=0, odd_frac=0.0)
    order = list(rng.permutation(nt))
    a = float(dense.koszul_value(tensors, bonds, order))
    b = dense.swap_gate_value(tensors, bonds, order)
    assert abs(a - b) <= 1e-12 * max(1.0, abs(a))


@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
@pytest.mark.parametrize("seed", range(5))
def test_local_even_independent_of_order(sym, seed):
    rng = np.random.default_rng(300 + seed)
    nt = int(rng.integers(2, 6))
    tensors, bonds = random_network(rng, sym, nt, nt + 1, n_open=0, odd_frac=0.0)
    vals = []
    for trial in range(3):
        order = list(rng.permutation(nt))
        vals.append(float(dense.koszul_value(tensors, bonds, order, local=True)))
    net = Network(tensors, bonds, conv="local")
    for trial in range(3):
        path = random_ssa_path(rng, tensors, bonds)
        T, labs, e = _value_with_open(net, path)
        vals.append(float(T.blocks.get((), 0.0)) * 2.0 ** e)
    for v in vals[1:]:
        assert abs(v - vals[0]) <= 1e-12 * max(1.0, abs(vals[0]))


@pytest.mark.parametrize("sym", [S.Z2, S.U1])
@pytest.mark.parametrize("seed", range(6))
def test_global_equals_local_after_dag_translation(sym, seed):
    # Sec. II.D/E: positions <-> DAG arrows; reversed arrows carry g; odd
    # tensors carry dummy legs sorted by position.
    rng = np.random.default_rng(400 + seed)
    nt = int(rng.integers(2, 6))
    tensors, bonds = random_network(rng, sym, nt, nt + 1, n_open=int(rng.integers(0, 2)),
                                    odd_frac=0.5)
    pos = list(rng.permutation(nt))
    order = sorted(range(nt), key=lambda t: pos[t])
    g = Network(tensors, bonds, conv="global", positions=pos)
    loc = to_local(g)
    path = random_ssa_path(rng, tensors, bonds)
    Tg, lg, eg = _value_with_open(g, path)
    Tl, ll, el = _value_with_open(loc, path)
    Tg = _to_flat_order(Tg, lg, order, tensors)
    Tl = _to_flat_order(Tl, ll, order, tensors)
    np.testing.assert_allclose(Tl.to_dense() * 2.0 ** el, Tg.to_dense() * 2.0 ** eg,
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_fused_bond_contraction_equals_separate(conv, sym):
    # Sec. IV.A: contracting over the fused bond equals contracting leg by leg
    rng = np.random.default_rng(500)
    for trial in range(6):
        m = int(rng.integers(2, 4))
        bond = [rand_leg(rng, sym) for _ in range(m)]
        fa = [rand_leg(rng, sym) for _ in range(2)]
        fb = [rand_leg(rng, sym) for _ in range(1)]
        A_legs = fa + bond
        B_legs = [partner(b) for b in bond] + fb
        pa = list(rng.permutation(len(A_legs)))
        pb = list(rng.permutation(len(B_legs)))
        A = rand_tensor(rng, sym, [A_legs[p] for p in pa], total=S.zero(sym))
        B = rand_tensor(rng, sym, [B_legs[p] for p in pb], total=S.zero(sym))
        ax_a = [pa.index(2 + t) for t in range(m)]
        ax_b = [pb.index(t) for t in range(m)]
        ref = ftensordot(A, B, ax_a, ax_b, conv)
        Af, _ = fuse(A, ax_a, conv=conv, rev=False)
        Bf, _ = fuse(B, ax_b, conv=conv, rev=True)
        ia = sum(1 for i in range(A.ndim) if i not in ax_a and i < ax_a[0])
        ib = sum(1 for i in range(B.ndim) if i not in ax_b and i < ax_b[0])
        got = ftensordot(Af, Bf, [ia], [ib], conv)
        np.testing.assert_allclose(got.to_dense(), ref.to_dense(), atol=1e-12)
