"""Pins of the oracle's derivatives (``oracle.adjoint``).

The derivatives come from reverse-mode differentiation of the oracle's
block arithmetic; they are pinned here by what the mathematics fixes:

* a pairwise contraction C(A, B) is bilinear (Eq. standardcontract), so for
  any cotangent dC: <dA, A> = <dC, C> = <dB, B>, and the directional
  difference L(A + V) - L(A - V) equals 2 <dA, V> exactly (up to rounding)
  for L(A) = <dC, C(A, B)>;
* the value of a closed network is linear in each tensor (Eq.
  fermionictn2): <grad_t, T_t> equals the value for every t (Euler's
  identity for degree-1 homogeneous functions), and the directional
  difference in T_t equals 2 <grad_t, V>;
* a gradient entry of a block the value does not depend on is zero.

A sign dropped or flipped in any block of the derivative changes one of
these sums.
"""

import numpy as np
import pytest

from oracle import symmetry as S
from oracle.adjoint import ftensordot_vjp, network_grad, inner
from oracle.ops import ftensordot
from oracle.network import Network, network_value
from tests.helpers import rand_leg, partner, rand_tensor, random_network, random_ssa_path

SYMS = [S.Z2, S.U1, S.U1U1]


def _pair(rng, sym, k, nfa, nfb, maxd=3):
    bond = [rand_leg(rng, sym, maxd=maxd) for _ in range(k)]
    fa = [rand_leg(rng, sym, maxd=maxd) for _ in range(nfa)]
    fb = [rand_leg(rng, sym, maxd=maxd) for _ in range(nfb)]
    A_legs, B_legs = fa + bond, [partner(b) for b in bond] + fb
    pa, pb = list(rng.permutation(len(A_legs))), list(rng.permutation(len(B_legs)))
    A = rand_tensor(rng, sym, [A_legs[p] for p in pa])
    B = rand_tensor(rng, sym, [B_legs[p] for p in pb])
    return A, B, [pa.index(nfa + t) for t in range(k)], [pb.index(t) for t in range(k)]


def _rel(x, y):
    return abs(float(x) - float(y)) / max(1.0, abs(float(y)))


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", SYMS)
def test_vjp_bilinear_identity_and_difference(sym, conv):
    rng = np.random.default_rng(11)
    for trial in range(6):
        A, B, ax_a, ax_b = _pair(rng, sym, int(rng.integers(0, 4)), int(rng.integers(0, 3)),
                                 int(rng.integers(0, 3)))
        C = ftensordot(A, B, ax_a, ax_b, conv=conv)
        dC = rand_tensor(rng, sym, C.legs, total=C.total)
        dA, dB = ftensordot_vjp(A, B, dC, ax_a, ax_b, conv)
        c = inner(dC, C)
        assert _rel(inner(dA, A), c) < 1e-12
        assert _rel(inner(dB, B), c) < 1e-12
        V = rand_tensor(rng, sym, A.legs, total=A.total)
        W = rand_tensor(rng, sym, B.legs, total=B.total)
        Ap = A.copy(); Am = A.copy()
        Bp = B.copy(); Bm = B.copy()
        for k in A.keys():
            Ap.blocks[k] = A.block(k) + V.block(k)
            Am.blocks[k] = A.block(k) - V.block(k)
        for k in B.keys():
            Bp.blocks[k] = B.block(k) + W.block(k)
            Bm.blocks[k] = B.block(k) - W.block(k)
        da = inner(dC, ftensordot(Ap, B, ax_a, ax_b, conv=conv)) - inner(dC, ftensordot(Am, B, ax_a, ax_b, conv=conv))
        db = inner(dC, ftensordot(A, Bp, ax_a, ax_b, conv=conv)) - inner(dC, ftensordot(A, Bm, ax_a, ax_b, conv=conv))
        assert _rel(da, 2 * inner(dA, V)) < 1e-12
        assert _rel(db, 2 * inner(dB, W)) < 1e-12


def test_vjp_sign_of_a_single_block():
    # Z2, one bond: C = A B with the local pairing sign on the odd sector when
    # A's end of the bond is '+'. Brute force per entry: dA[i, k] = sum_j
    # dC[i, j] * sign(k) * B[k, j], the sign being -1 on the odd sector only.
    from oracle.tensor import make_leg
    rng = np.random.default_rng(12)
    lf = make_leg(S.Z2, [(0,), (1,)], [2, 3], 0)
    lb = make_leg(S.Z2, [(0,), (1,)], [2, 2], 0)
    A = rand_tensor(rng, S.Z2, [lf, lb], total=(0,))
    B = rand_tensor(rng, S.Z2, [partner(lb), partner(lf)], total=(0,))
    C = ftensordot(A, B, [1], [0], conv="local")
    dC = rand_tensor(rng, S.Z2, C.legs, total=C.total)
    dA, _ = ftensordot_vjp(A, B, dC, [1], [0], "local")
    a = A.to_dense(); b = B.to_dense(); dc = dC.to_dense()
    sgn = np.array([1, 1, -1, -1.0])
    ref = dc @ (sgn[:, None] * b).T
    mask = np.zeros_like(ref)
    for k in A.keys():
        sl = tuple(slice(l.offset(i), l.offset(i) + l.dims[i]) for l, i in zip(A.legs, k))
        mask[sl] = 1
    np.testing.assert_allclose(dA.to_dense(), ref * mask, rtol=0, atol=1e-12)


def _networks(sym, n, count):
    rng = np.random.default_rng(13)
    out = []
    while len(out) < count:
        tensors, bonds = random_network(rng, sym, n, n + 2, odd_frac=0.4)
        if sum(tensors[t].parity for t in tensors) % 2:
            continue
        path = random_ssa_path(rng, tensors, bonds)
        net = Network(tensors, bonds, conv="local", positions=list(rng.permutation(n)))
        if abs(network_value(net, path)[0]) < 1e-3:
            continue
        out.append((net, path, rng))
    return out


@pytest.mark.parametrize("sym", [S.Z2, S.U1])
def test_network_grad_euler_and_difference(sym):
    for net, path, rng in _networks(sym, 5, 3):
        v, g = network_grad(net, path)
        for t, T in net.tensors.items():
            assert _rel(inner(g[t], T), v) < 1e-11
            V = rand_tensor(rng, sym, T.legs, total=T.total)
            vals = []
            for s in (1.0, -1.0):
                X = T.copy()
                for k in T.keys():
                    X.blocks[k] = T.block(k) + s * V.block(k)
                tens = dict(net.tensors)
                tens[t] = X
                m, e = network_value(Network(tens, net.bonds, conv="local", positions=net.positions), path)
                vals.append(m * 2.0 ** e)
            assert _rel(vals[0] - vals[1], 2 * inner(g[t], V)) < 1e-11


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1])
def test_compress_product_grad_directional_difference(sym, conv):
    # L = <W, F(A' B')> is unchanged by the sign of each kept singular vector
    # pair, so its derivative through the truncated SVD is well defined; a
    # central difference (kept counts unchanged) must agree with it
    from oracle.linalg import compress_bond
    from oracle.adjoint import compress_product_grad
    rng = np.random.default_rng(14)
    for trial in range(3):
        bond = rand_leg(rng, sym, maxd=5)
        A = rand_tensor(rng, sym, [rand_leg(rng, sym, maxd=3), bond, rand_leg(rng, sym, maxd=3)],
                        total=S.zero(sym))
        B = rand_tensor(rng, sym, [partner(bond), rand_leg(rng, sym, maxd=3)], total=S.zero(sym))
        chi = int(rng.integers(2, 5))

        def loss(A_, B_, W):
            A2, B2, _ = compress_bond(A_, B_, 1, 0, chi, conv=conv, cutoff=1e-6)
            return inner(W, ftensordot(A2, B2, [1], [0], conv=conv)), A2, B2

        A2, B2, _ = compress_bond(A, B, 1, 0, chi, conv=conv, cutoff=1e-6)
        C = ftensordot(A2, B2, [1], [0], conv=conv)
        W = rand_tensor(rng, sym, C.legs, total=C.total)
        gA, gB = compress_product_grad(A, B, 1, 0, chi, W, conv=conv)
        V = rand_tensor(rng, sym, A.legs, total=A.total)
        h = 1e-6
        Ap, Am = A.copy(), A.copy()
        for k in A.keys():
            Ap.blocks[k] = A.block(k) + h * V.block(k)
            Am.blocks[k] = A.block(k) - h * V.block(k)
        fd = (float(loss(Ap, B, W)[0]) - float(loss(Am, B, W)[0])) / (2 * h)
        an = float(inner(gA, V))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_network_grad_with_compression_rank_deficient_factors():
    # compressions whose factors are rank deficient (a one-row factor, bonds
    # of rank one): the oracle's derivative must still agree with central
    # differences of the compressed network value
    from tests.helpers import random_network, random_ssa_path
    rng = np.random.default_rng(741)
    while True:
        nt = int(rng.integers(4, 7))
        tensors, bonds = random_network(rng, S.Z2, nt, nt + 3, odd_frac=0.5, maxd=3)
        if sum(tensors[t].parity for t in tensors) % 2:
            continue
        pos = [int(x) for x in rng.permutation(nt)]
        path = random_ssa_path(rng, tensors, bonds)
        from oracle.network import contract_network
        T, _, _, infos = contract_network(Network(tensors, bonds, conv="local", positions=pos), path, chi=3)
        if () in T.blocks and float(T.blocks[()]) != 0.0 and infos:
            break
    net = Network(tensors, bonds, conv="local", positions=pos)
    v, g = network_grad(net, path, chi=3)
    r2 = np.random.default_rng(5)
    for t in range(nt):
        V = rand_tensor(r2, S.Z2, tensors[t].legs, total=tensors[t].total)
        vals = []
        for h in (1e-5, -1e-5):
            X = tensors[t].copy()
            for k in X.keys():
                X.blocks[k] = tensors[t].block(k) + h * V.block(k)
            tt = dict(tensors)
            tt[t] = X
            m, e = network_value(Network(tt, bonds, conv="local", positions=pos), path, chi=3)
            vals.append(m * 2.0 ** e)
        fd = (vals[0] - vals[1]) / 2e-5
        an = float(inner(g[t], V))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)


def _hubbard_setup(shape, d, seed):
    from oracle import physics as OP
    from oracle.tensor import FTensor
    from synth import workloads as W
    from synth.graphs import square_lattice
    from synth.operators import operator_dense
    n, edges = square_lattice(*shape)
    spec = W.z2_peps(n, edges, *d)
    rng = np.random.default_rng(seed)
    kets = OP.ket_tensors(spec, [rng.standard_normal(s.dense_shape) for s in spec.sites])
    phys = kets[0].legs[0]
    from oracle.tensor import Leg
    out_l, in_l = phys, Leg(phys.charges, phys.dims, 1)
    terms = []
    for kind, sites in W.hubbard_terms(spec):
        G = FTensor.from_dense(S.Z2, [out_l, out_l, in_l, in_l], (0,), operator_dense(kind, "Z2"))
        terms.append((G, sites))
    paths = {None: W.norm_path(spec, seed=1)}
    for _, sites in terms:
        paths[tuple(sites)] = W.norm_path(spec, seed=1, op_sites=tuple(sites))
    return spec, kets, terms, paths


@pytest.mark.parametrize("chi", [None, 4])
def test_energy_gradient_directional_difference(chi):
    from oracle.adjoint import energy_grad
    from oracle import physics as OP
    from oracle.network import contract_network
    spec, kets, terms, paths = _hubbard_setup((2, 2), (2, 1), 33)
    E, grads = energy_grad(spec, kets, terms, paths, chi=chi)

    def energy(ks):
        def value(op=None, sites=None):
            net = OP.norm_network(spec, ks, op=op, op_sites=sites, conv="local")
            T, _, e, _ = contract_network(net, paths[None if op is None else tuple(sites)], chi=chi)
            return (float(T.blocks[()]) if () in T.blocks else 0.0) * 2.0 ** e
        return sum(value(G, s) for G, s in terms) / value()

    assert abs(energy(kets) - E) <= 1e-10 * abs(E)
    rng = np.random.default_rng(34)
    for s in (0, 3):
        V = rand_tensor(rng, S.Z2, kets[s].legs, total=kets[s].total)
        vals = []
        for h in (1e-5, -1e-5):
            X = kets[s].copy()
            for k in X.keys():
                X.blocks[k] = kets[s].block(k) + h * V.block(k)
            ks = list(kets)
            ks[s] = X
            vals.append(energy(ks))
        fd = (vals[0] - vals[1]) / 2e-5
        an = float(inner(grads[s], V))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (s, fd, an)
