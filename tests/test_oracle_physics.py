"""Physics pins of the oracle: Jordan-Wigner exact diagonalisation (CPU).

The ket network with open physical legs is the coefficient tensor of the
state in the Jordan-Wigner basis; the norm network (Fig. 4a) must give the
sum of squares, and with a two-site operator tensor inserted it must give
the Fock-space expectation value of that term (Eq. fermi-hubbard-ham),
whether or not the two sites are adjacent in the mode order. The variational
energy is bounded below by the ground-state energy (scipy eigsh).
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import symmetry as S, dense, physics as P
from oracle.network import Network, contract_network, network_value, to_local
from oracle.ops import ftranspose
from synth import workloads as W
from synth.graphs import square_lattice


def _psi(spec, kets):
    kn = P.ket_network(spec, kets)
    return dense.koszul_value(kn.tensors, kn.bonds, list(range(spec.n_sites)))


def _val(net, path, chi=None):
    m, e = network_value(net, path, chi=chi)
    return m * 2.0 ** e


@pytest.mark.parametrize("shape,d", [((2, 2), (1, 1)), ((2, 3), (1, 1)), ((2, 2), (2, 1))])
def test_norm_and_terms_match_ed(shape, d):
    n, edges = square_lattice(*shape)
    spec = W.z2_peps(n, edges, *d)
    rng = np.random.default_rng(30)
    vals = [rng.standard_normal(s.dense_shape) for s in spec.sites]
    kets = P.ket_tensors(spec, vals)
    psi = _psi(spec, kets)
    fv = P.psi_to_fock(psi, S.Z2)
    nrm = float(fv @ fv)
    path = W.norm_path(spec, seed=1)
    for conv in ("global", "local"):
        net = P.norm_network(spec, kets, conv=conv)
        assert abs(_val(net, path) - nrm) <= 1e-10 * nrm
    phys = kets[0].legs[0]
    terms = [("hop", e) for e in edges] + [("hop", (0, n - 1))]
    for kind, (u, v) in terms:
        G = P.operator_tensor(P.two_site_local(kind), phys, S.Z2)
        h = P.hopping_term(n, u, v)
        ref = float(fv @ (h @ fv))
        p2 = W.norm_path(spec, seed=2, op_sites=(u, v))
        for conv in ("global", "local"):
            net = P.norm_network(spec, kets, op=G, op_sites=(u, v), conv=conv)
            got = _val(net, p2)
            assert abs(got - ref) <= 1e-10 * nrm, (kind, u, v, conv, got, ref)
    # on-site U via a two-site tensor with identity on the partner
    for u in range(n):
        v = (u + 1) % n
        a, b = min(u, v), max(u, v)
        h16 = P.two_site_local("nn_u")
        if u == b:
            # n_up n_dn on the second site of the pair: swap the mode blocks
            idx = np.arange(16)
            perm = ((idx & 3) << 2) | (idx >> 2)
            h16 = h16[np.ix_(perm, perm)]
        G = P.operator_tensor(h16, phys, S.Z2)
        ref = float(fv @ (P.onsite_term(n, u, U=1.0) @ fv))
        net = P.norm_network(spec, kets, op=G, op_sites=(a, b), conv="local")
        got = _val(net, W.norm_path(spec, seed=3, op_sites=(a, b)))
        assert abs(got - ref) <= 1e-10 * nrm


def test_energy_above_ground_state():
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    rng = np.random.default_rng(31)
    vals = [rng.standard_normal(s.dense_shape) for s in spec.sites]
    kets = P.ket_tensors(spec, vals)
    fv = P.psi_to_fock(_psi(spec, kets), S.Z2)
    H = P.hubbard(n, edges, t=1.0, U=8.0)
    e0 = spla.eigsh(H, k=1, which="SA")[0][0]
    e = float(fv @ (H @ fv)) / float(fv @ fv)
    assert e >= e0 - 1e-10


def test_u1u1_toy_norm_and_hopping():
    # U(1)xU(1) 2x2 toy (reading: parity = (n_up + n_dn) mod 2)
    from synth.peps import make_peps, u1u1_leg, U1U1
    n, edges = square_lattice(2, 2)
    phys = {(0, 0): 1, (0, 1): 1, (1, 0): 1, (1, 1): 1}
    bond = {(0, 0): 1, (1, 0): 1, (-1, 0): 1, (0, 1): 1, (0, -1): 1}
    spec = make_peps(U1U1, n, edges, lambda: u1u1_leg(phys, 0),
                     lambda dual: u1u1_leg(bond, dual),
                     lambda s: (1, 1) if s % 2 == 0 else (0, 0))
    rng = np.random.default_rng(32)
    vals = [rng.standard_normal(s.dense_shape) for s in spec.sites]
    kets = P.ket_tensors(spec, vals)
    psi = _psi(spec, kets)
    fv = P.psi_to_fock(psi, S.U1U1)
    nrm = float(fv @ fv)
    assert nrm > 0
    path = W.norm_path(spec, seed=1)
    assert abs(_val(P.norm_network(spec, kets, conv="local"), path) - nrm) <= 1e-10 * nrm
    G = P.operator_tensor(P.two_site_local("hop"), kets[0].legs[0], S.U1U1)
    for (u, v) in edges:
        ref = float(fv @ (P.hopping_term(n, u, v) @ fv))
        net = P.norm_network(spec, kets, op=G, op_sites=(u, v), conv="local")
        got = _val(net, W.norm_path(spec, seed=2, op_sites=(u, v)))
        assert abs(got - ref) <= 1e-10 * nrm


def test_odd_parity_amplitude_is_zero():
    # an even-parity PEPS has zero amplitude on odd-parity configurations
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    rng = np.random.default_rng(33)
    kets = P.ket_tensors(spec, [rng.standard_normal(s.dense_shape) for s in spec.sites])
    psi = _psi(spec, kets)
    for idx in np.ndindex(*psi.shape):
        if sum(i >= 2 for i in idx) % 2:
            assert psi[idx] == 0.0


def test_approximate_limit_is_exact():
    # chi above every bond's exact rank: approximate contraction is exact
    cfg = W.c2(n_sites=8, chi=10 ** 6)
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"])
    kets = P.ket_tensors(spec, vals)
    net = P.norm_network(spec, kets, conv="local")
    path = W.norm_path(spec, chi=None, seed=0)
    exact = _val(net, path)
    approx = _val(net, path, chi=10 ** 6)
    assert abs(approx - exact) <= 1e-12 * abs(exact)
    # a moderate chi stays close; the global convention gives the same value
    a_loc = _val(net, path, chi=64)
    a_glo = _val(P.norm_network(spec, kets, conv="global"), path, chi=64)
    assert abs(a_loc - a_glo) <= 1e-10 * abs(a_loc)


def _padded_site_values(spec, spec_big, vals, rng):
    """Site values of the same state with every bond sector widened.

    For each bond (i, j), i < j, a random per-sector map E (d x d') with a
    right inverse E+ (E E+ = 1) is applied to the bond leg of site i (E) and
    of site j (E+). Sectors keep their parity, so every fermionic sign of the
    contraction over the bond is unchanged and the network value is that of
    the unpadded state; the bond dimension grows but the rank across it does
    not.
    """
    out = [v.copy() for v in vals]
    for (i, j) in spec.edges:
        li, lj = spec.bond_leg(i, j), spec.bond_leg(j, i)
        small = spec.sites[i].legs[li]
        big = spec_big.sites[i].legs[li]
        E = np.zeros((small.size, big.size))
        o_s = o_b = 0
        for d, db in zip(small.dims, big.dims):
            E[o_s:o_s + d, o_b:o_b + db] = rng.standard_normal((d, db))
            o_s += d
            o_b += db
        Ep = np.linalg.pinv(E)                      # E @ Ep = 1 (full row rank)
        out[i] = np.moveaxis(np.tensordot(out[i], E, axes=([li], [0])), -1, li)
        out[j] = np.moveaxis(np.tensordot(out[j], Ep.T, axes=([lj], [0])), -1, lj)
    return out


def test_approximate_limit_with_compression_is_exact():
    # bonds (1|1) widened to (2|2): a fused bra-ket bond is 16 wide but of
    # rank 4 (the unpadded 2 x 2), so with chi = 8 every such bond is
    # compressed while chi stays at or above the exact rank across every cut
    # the path meets: the approximate contraction must reproduce the exact
    # value, through compress_bond, with nothing but zeros discarded
    n, edges = square_lattice(2, 3)
    spec = W.z2_peps(n, edges, 1, 1)
    big = W.z2_peps(n, edges, 2, 2)
    rng = np.random.default_rng(140)
    vals = [rng.standard_normal(s.dense_shape) for s in spec.sites]
    pv = _padded_site_values(spec, big, vals, rng)
    exact = _val(P.norm_network(spec, P.ket_tensors(spec, vals), conv="local"), W.norm_path(spec, seed=0))
    net = P.norm_network(big, P.ket_tensors(big, pv), conv="local")
    path = W.norm_path(big, seed=0)
    assert abs(_val(net, path) - exact) <= 1e-12 * abs(exact)
    T, _, e, infos = contract_network(net, path, chi=8)
    truncating = [i for i in infos if len(i["all_svals"]) > sum(len(v) for v in i["svals"].values())]
    assert len(truncating) >= 3                            # compression ran and cut
    for i in truncating:
        assert i["discarded"] <= 1e-24 * i["total"]        # only zero values dropped
    approx = float(T.blocks[()]) * 2.0 ** e
    assert abs(approx - exact) <= 1e-12 * abs(exact), (approx, exact)
    # a chi below the exact rank is no longer exact
    T2, _, e2, _ = contract_network(net, path, chi=2)
    assert abs(float(T2.blocks[()]) * 2.0 ** e2 - exact) > 1e-6 * abs(exact)
