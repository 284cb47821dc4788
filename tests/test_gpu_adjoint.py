"""GPU parity of the adjoint contraction and of network gradients.

``ftensordot_backward`` (C ABI) is compared block by block with the
oracle's reverse-mode derivative of its own contraction; the structures of
dA and dB (the structures of A and B) must match bit-exactly. FP64 values
agree up to summation order: each cotangent entry is a dot product of
length N (dA) or M (dB) of O(1) terms, checked as a max error of 1e-12
relative to the largest entry. Network gradients go through the autograd
driver (every contraction and transposition in the library) and are
compared with the oracle's gradient of the exact network value at 1e-11
relative (a few chained FP64 contractions).
"""

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from oracle.adjoint import ftensordot_vjp, network_grad, inner
from oracle.network import Network, network_value
from oracle.ops import ftensordot
from oracle.tensor import make_leg
from tests.helpers import rand_leg, partner, rand_tensor, random_network, random_ssa_path
from tests.gpu_helpers import to_gpu, assert_same_structure, flat_blocks, legs_abi, SYM
from tests.test_gpu_ops import _rand_pair

pytestmark = pytest.mark.gpu

SYMS = [S.Z2, S.U1, S.U1U1]


@pytest.fixture(scope="module")
def P():
    import paper_2410_02215_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    P.load_library()
    return P


def _data(G):
    return G.data().double().cpu().numpy()


def _check(ref, G, tol):
    assert_same_structure(ref, G)
    r = flat_blocks(ref)
    err = np.abs(_data(G) - r).max(initial=0)
    assert err <= tol * max(1.0, np.abs(r).max(initial=0)), err


def _backward_case(P, A, B, ax_a, ax_b, conv, rng, dtype=torch.float64, gemm=None, tol=1e-12):
    ref_c = ftensordot(A, B, ax_a, ax_b, conv=conv)
    dC = rand_tensor(rng, A.sym, ref_c.legs, total=ref_c.total)
    dA, dB = ftensordot_vjp(A, B, dC, ax_a, ax_b, conv)
    c = P.LOCAL if conv == "local" else P.GLOBAL
    g = P.GEMM_F64 if gemm is None else gemm
    GdA, GdB = P.ftensordot_backward(to_gpu(A, dtype), to_gpu(B, dtype), to_gpu(dC, dtype), ax_a, ax_b,
                                     conv=c, gemm=g)
    _check(dA, GdA, tol)
    _check(dB, GdB, tol)


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", SYMS)
def test_ftensordot_backward_fp64(P, sym, conv):
    rng = np.random.default_rng(21)
    for trial in range(8):
        k = int(rng.integers(0, 4))
        A, B, ax_a, ax_b = _rand_pair(rng, sym, k, int(rng.integers(0, 4)), int(rng.integers(0, 4)), 3)
        _backward_case(P, A, B, ax_a, ax_b, conv, rng)


def test_ftensordot_backward_tiles_and_ragged_tails(P):
    # sectors spanning several GEMM tiles in every role (M, N and K of both
    # adjoint products) with ragged edges
    rng = np.random.default_rng(22)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rand_tensor(rng, sym, [l(37, 141, 0), l(70, 9, 1), l(213, 30, 0)], total=(0,))
    B = rand_tensor(rng, sym, [l(213, 30, 1), l(150, 3, 0)], total=(1,))
    _backward_case(P, A, B, [2], [0], "local", rng)
    _backward_case(P, A, B, [2], [0], "global", rng)


def test_ftensordot_backward_scalar_output(P):
    # full contraction of two tensors: C is one number, dA = dC * B (signed)
    rng = np.random.default_rng(23)
    sym = S.U1
    l = lambda d: make_leg(sym, [(-1,), (0,), (1,)], [2, 3, 1], d)
    A = rand_tensor(rng, sym, [l(0), l(1), l(0)], total=(0,))
    B = rand_tensor(rng, sym, [l(1), l(0), l(1)], total=(0,))
    _backward_case(P, A, B, [0, 1, 2], [2, 1, 0], "local", rng)
    _backward_case(P, A, B, [2, 0, 1], [0, 2, 1], "global", rng)


@pytest.mark.parametrize("gemm", ["f32", "bf16x3"])
def test_ftensordot_backward_fp32_forms(P, gemm):
    rng = np.random.default_rng(24)
    g = P.GEMM_F32 if gemm == "f32" else P.GEMM_BF16X3
    tol = {"f32": 1e-5, "bf16x3": 1e-4}[gemm]
    for trial in range(4):
        A, B, ax_a, ax_b = _rand_pair(rng, S.U1U1, int(rng.integers(1, 3)), 2, 2, 4)
        _backward_case(P, A, B, ax_a, ax_b, "local", rng, dtype=torch.float32, gemm=g, tol=tol)


def test_ftensordot_backward_rejects_wrong_cotangent(P):
    rng = np.random.default_rng(25)
    A, B, ax_a, ax_b = _rand_pair(rng, S.Z2, 1, 2, 1, 3)
    with pytest.raises(P.FtnError) as e:
        P.ftensordot_backward(to_gpu(A), to_gpu(B), to_gpu(B), ax_a, ax_b)
    assert e.value.code == -1


def _dtensor(T):
    from paper_2410_02215_amd.autograd import DTensor
    G = to_gpu(T)
    d = G.data()
    d.requires_grad_(True)
    tot = tuple(T.total) + ((0,) if len(T.total) == 1 else ())
    return DTensor(SYM[T.sym], legs_abi(T.legs), tot, d)


@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_network_gradient_matches_oracle(P, sym):
    from paper_2410_02215_amd import autograd as AG
    rng = np.random.default_rng(26)
    done = 0
    while done < 3:
        n = int(rng.integers(3, 7))
        tensors, bonds = random_network(rng, sym, n, n + 2, odd_frac=0.4)
        if sum(tensors[t].parity for t in tensors) % 2:
            continue
        path = random_ssa_path(rng, tensors, bonds)
        order = [int(x) for x in rng.permutation(n)]
        net = Network(tensors, bonds, conv="local", positions=order)
        v, grads = network_grad(net, path)
        if abs(v) < 1e-3:
            continue
        D = [_dtensor(tensors[t]) for t in range(n)]
        val = AG.network_value(D, bonds, path, order=order)
        assert abs(float(val.detach()) - v) <= 1e-11 * max(1.0, abs(v))
        gs = torch.autograd.grad(val, [d.data for d in D])
        for t in range(n):
            r = flat_blocks(grads[t])
            err = np.abs(gs[t].double().cpu().numpy() - r).max(initial=0)
            assert err <= 1e-11 * max(1.0, np.abs(r).max(initial=0)), (t, err)
        # exact contraction through the library's backward pass (odd tensors:
        # the dummy-leg sign is part of the seed)
        gnet = P.Network([to_gpu(tensors[t]) for t in range(n)], bonds, conv=P.LOCAL, positions=order)
        m2, e2n, ng = gnet.contract_grad(path, chi=0, checkpoint=1)
        assert abs(m2 * 2.0 ** e2n - v) <= 1e-11 * max(1.0, abs(v))
        for t in range(n):
            r = flat_blocks(grads[t])
            err = np.abs(ng[t].data().cpu().numpy() * 2.0 ** e2n - r).max(initial=0)
            assert err <= 1e-11 * max(1.0, np.abs(r).max(initial=0)), (t, err)
        done += 1


def _compress_case(P, A, B, la, lb, chi, conv, rng):
    from oracle.linalg import compress_bond as o_compress
    from oracle.adjoint import compress_product_grad
    A2, B2, _ = o_compress(A, B, la, lb, chi, conv=conv, cutoff=1e-6)
    C = ftensordot(A2, B2, [la], [lb], conv=conv)
    W = rand_tensor(rng, A.sym, C.legs, total=C.total)
    gA, gB = compress_product_grad(A, B, la, lb, chi, W, conv=conv)
    cv = P.LOCAL if conv == "local" else P.GLOBAL
    ga, gb = to_gpu(A), to_gpu(B)
    GA, GB, _ = P.compress_bond(ga, gb, la, lb, chi, 1e-6, cv)
    dGA, dGB = P.ftensordot_backward(GA, GB, to_gpu(W), [la], [lb], conv=cv)
    da, db = P.compress_bond_backward(ga, gb, la, lb, chi, dGA, dGB, 1e-6, cv)
    # the loss depends on the compressed pair only through its product, so
    # the gradient does not depend on either side's sign choices
    _check(gA, da, 1e-8)
    _check(gB, db, 1e-8)


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", SYMS)
def test_compress_bond_backward_matches_oracle(P, sym, conv):
    rng = np.random.default_rng(27)
    for trial in range(4):
        bond = rand_leg(rng, sym, maxd=6)
        la_ = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        lb_ = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        pa, pb = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        A = rand_tensor(rng, sym, la_[:pa] + [bond] + la_[pa:], total=S.zero(sym))
        B = rand_tensor(rng, sym, lb_[:pb] + [partner(bond)] + lb_[pb:], total=S.zero(sym))
        _compress_case(P, A, B, pa, pb, int(rng.integers(2, 8)), conv, rng)


def test_compress_bond_backward_tall_factors_and_odd_tensors(P):
    # sectors with many more rows than columns (shifted Cholesky QR), odd
    # tensors, and a bond dimension of 60 per sector
    rng = np.random.default_rng(28)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rand_tensor(rng, sym, [l(20, 17, 0), l(30, 30, 1), l(9, 8, 0)], total=(1,))
    B = rand_tensor(rng, sym, [l(30, 30, 0), l(25, 33, 1)], total=(0,))
    _compress_case(P, A, B, 1, 0, 24, "local", rng)


@pytest.mark.parametrize("dims", [((200, 200), (130, 2), (150, 150)),      # one sector just above 128
                                  ((300, 280), (256, 256), (280, 300)),    # 256 in both sectors
                                  ((90, 120), (200, 40), (260, 50))])     # fewer rows than the sector (rank 90)
def test_compress_bond_backward_large_sectors(P, dims):
    # bond sectors above 128: eigenpairs by block Jacobi, factors by the
    # blocked Cholesky with its inverse
    rng = np.random.default_rng(29)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    (ae, ao), (be, bo), (ce, co) = dims
    A = rand_tensor(rng, sym, [l(ae, ao, 0), l(be, bo, 1)], total=(0,))
    B = rand_tensor(rng, sym, [l(be, bo, 0), l(ce, co, 1)], total=(0,))
    _compress_case(P, A, B, 1, 0, 24, "local", rng)


def test_compress_bond_backward_large_and_small_u1_sectors(P):
    rng = np.random.default_rng(31)
    sym = S.U1
    q = [(-1,), (0,), (1,)]
    bond = make_leg(sym, q, [140, 40, 150], 0)
    A = rand_tensor(rng, sym, [make_leg(sym, q, [150, 70, 160], 1), make_leg(sym, q, [1, 2, 1], 0), bond],
                    total=(0,))
    B = rand_tensor(rng, sym, [partner(bond), make_leg(sym, q, [160, 80, 170], 1)], total=(0,))
    _compress_case(P, A, B, 2, 0, 40, "global", rng)


def test_autograd_compress_then_contract(P):
    from paper_2410_02215_amd import autograd as AG
    from oracle.linalg import compress_bond as o_compress
    from oracle.adjoint import compress_product_grad
    rng = np.random.default_rng(30)
    sym = S.U1
    bond = make_leg(sym, [(-1,), (0,), (1,)], [3, 5, 4], 0)
    A = rand_tensor(rng, sym, [make_leg(sym, [(-1,), (0,), (1,)], [2, 3, 2], 1), bond], total=(0,))
    B = rand_tensor(rng, sym, [partner(bond), make_leg(sym, [(-1,), (0,), (1,)], [2, 2, 3], 0)], total=(0,))
    chi = 5
    A2, B2, _ = o_compress(A, B, 1, 0, chi, conv="local", cutoff=1e-6)
    C = ftensordot(A2, B2, [1], [0], conv="local")
    W = rand_tensor(rng, sym, C.legs, total=C.total)
    gA, gB = compress_product_grad(A, B, 1, 0, chi, W, conv="local")
    a, b = _dtensor(A), _dtensor(B)
    a2, b2 = AG.compress(a, b, 1, 0, chi)
    c = AG.dot(a2, b2, [1], [0])
    w = to_gpu(W).data()
    loss = (c.data * w).sum()
    da, db = torch.autograd.grad(loss, [a.data, b.data])
    for g_ref, g in ((gA, da), (gB, db)):
        r = flat_blocks(g_ref)
        err = np.abs(g.double().cpu().numpy() - r).max(initial=0)
        assert err <= 1e-8 * max(1.0, np.abs(r).max(initial=0)), err


def _net_grad_case(P, tensors, bonds, path, pos, chi, tol):
    from paper_2410_02215_amd import autograd as AG
    n = len(tensors)
    net = Network(tensors, bonds, conv="local", positions=pos)
    v, grads = network_grad(net, path, chi=chi)
    D = [_dtensor(tensors[t]) for t in range(n)]
    F, labs, e2 = AG.contract(D, bonds, path, chi=chi, order=pos)
    assert F.ndim == 0
    val = F.data.sum()
    got = float(val.detach()) * 2.0 ** e2
    assert abs(got - v) <= tol * max(abs(v), 1e-300), (got, v)
    # the library's own driver takes the same steps
    m, e, _ = P.Network([to_gpu(tensors[t]) for t in range(n)], bonds, conv=P.LOCAL, positions=pos).contract(path, chi=chi or 0)
    assert abs(m * 2.0 ** e - got) <= 1e-13 * abs(got)
    gs = torch.autograd.grad(val, [d.data for d in D])
    for t in range(n):
        r = flat_blocks(grads[t])
        g = gs[t].double().cpu().numpy() * 2.0 ** e2
        err = np.abs(g - r).max(initial=0)
        assert err <= tol * max(1e-300, np.abs(r).max(initial=0)), (t, err, np.abs(r).max(initial=0))
    # the library's own backward pass, keeping every intermediate and with
    # recomputation segments of two path steps
    gnet = P.Network([to_gpu(tensors[t]) for t in range(n)], bonds, conv=P.LOCAL, positions=pos)
    for ck in (0, 2):
        m2, e2n, ng = gnet.contract_grad(path, chi=chi or 0, checkpoint=ck)
        assert abs(m2 * 2.0 ** e2n - v) <= tol * max(abs(v), 1e-300), (ck, m2 * 2.0 ** e2n, v)
        for t in range(n):
            r = flat_blocks(grads[t])
            g = ng[t].data().cpu().numpy() * 2.0 ** e2n
            err = np.abs(g - r).max(initial=0)
            assert err <= tol * max(1e-300, np.abs(r).max(initial=0)), (ck, t, err, np.abs(r).max(initial=0))


@pytest.mark.parametrize("seed", range(3))
def test_approximate_network_gradient_matches_oracle(P, seed):
    # odd tensors, parallel bonds fused and compressed at chi = 3
    rng = np.random.default_rng(740 + seed)
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
    _net_grad_case(P, tensors, bonds, path, pos, 3, 1e-7)


def test_peps_norm_gradient_with_compression(P):
    from oracle import physics as OP
    from synth import workloads as W
    from synth.graphs import square_lattice
    n, edges = square_lattice(2, 3)
    spec = W.z2_peps(n, edges, 2, 2)
    rng = np.random.default_rng(31)
    kets = OP.ket_tensors(spec, [rng.standard_normal(s.dense_shape) for s in spec.sites])
    net = OP.norm_network(spec, kets, conv="local")
    path = W.norm_path(spec, seed=1)
    tensors = [net.tensors[t] for t in range(2 * n)]
    _net_grad_case(P, tensors, net.bonds, path, net.positions, 6, 1e-7)


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1])
def test_fuse_backward_matches_oracle(P, sym, conv):
    from oracle.ops import fuse as o_fuse
    from oracle.adjoint import _leaf_copy
    rng = np.random.default_rng(32)
    for trial in range(6):
        n = int(rng.integers(2, 5))
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        m = int(rng.integers(1, n + 1))
        gl = [int(x) for x in rng.permutation(n)[:m]]
        rev = int(rng.integers(0, 2))
        T1 = _leaf_copy(T)
        F, _ = o_fuse(T1, gl, conv=conv, rev=rev)
        W = rand_tensor(rng, sym, F.legs, total=F.total)
        L = inner(W, F)
        keys = T1.keys()
        gs = torch.autograd.grad(L, [T1.blocks[k] for k in keys], allow_unused=True) if torch.is_tensor(L) and L.requires_grad else [None] * len(keys)
        ref = np.concatenate([np.zeros(T1.blocks[k].numel()) if g is None else g.numpy().ravel() for k, g in zip(keys, gs)]) if keys else np.zeros(0)
        c = P.LOCAL if conv == "local" else P.GLOBAL
        G = to_gpu(T)
        got = P.fuse_backward(G, gl, to_gpu(W), conv=c, rev=rev).data().double().cpu().numpy()
        np.testing.assert_array_equal(got, ref)


def test_exact_gradient_of_a_network_with_fused_bonds(P):
    # the same small network contracted exactly and with chi = 3
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
    _net_grad_case(P, tensors, bonds, path, pos, None, 1e-10)


@pytest.mark.parametrize("shape,d,chi", [((2, 2), (2, 1), None), ((2, 3), (2, 2), 6)])
def test_hubbard_energy_gradient_matches_oracle(P, shape, d, chi):
    from paper_2410_02215_amd import autograd as AG
    from paper_2410_02215_amd import peps as GP
    from oracle.adjoint import energy_grad
    from synth import workloads as W
    from synth.operators import operator_dense
    from tests.test_oracle_adjoint import _hubbard_setup
    spec, kets, terms, paths = _hubbard_setup(shape, d, 35)
    E, grads = energy_grad(spec, kets, terms, paths, chi=chi)
    D = [_dtensor(k) for k in kets]
    gterms = [(AG.DTensor.from_tensor(GP.operator_tensor(spec, operator_dense(kind, "Z2"))), sites)
              for kind, sites in W.hubbard_terms(spec)]
    Eg = AG.expectation_ratio(spec, D, gterms, paths, chi=chi)
    assert abs(float(Eg.detach()) - E) <= 1e-9 * abs(E)
    gs = torch.autograd.grad(Eg, [x.data for x in D])
    for s in range(len(kets)):
        r = flat_blocks(grads[s])
        err = np.abs(gs[s].double().cpu().numpy() - r).max(initial=0)
        assert err <= 1e-7 * max(1e-300, np.abs(r).max(initial=0)), (s, err)
    # the library's backward pass per network, combined by ftn_tensor_axpy,
    # with every intermediate kept and with recomputation segments of 3 steps
    gk = [to_gpu(k) for k in kets]
    gops = [(GP.operator_tensor(spec, operator_dense(kind, "Z2")), sites) for kind, sites in W.hubbard_terms(spec)]
    for ck in (0, 3):
        En, gn = GP.energy_gradient(spec, gk, gops, paths, chi=chi or 0, checkpoint=ck)
        assert abs(En - E) <= 1e-9 * abs(E), (ck, En, E)
        for s in range(len(kets)):
            r = flat_blocks(grads[s])
            err = np.abs(gn[s].data().cpu().numpy() - r).max(initial=0)
            assert err <= 1e-7 * max(1e-300, np.abs(r).max(initial=0)), (ck, s, err)


@pytest.mark.parametrize("ck", [1, 4])
def test_checkpointed_energy_gradient_matches_the_stored_one(P, ck):
    # recomputation checkpoints change what is stored, not what is computed:
    # the same value (bitwise: the forward kernels see the same inputs) and
    # the same gradient up to the order in which contributions are summed
    from paper_2410_02215_amd import autograd as AG
    from paper_2410_02215_amd import peps as GP
    from synth import workloads as W
    from synth.operators import operator_dense
    from tests.test_oracle_adjoint import _hubbard_setup
    spec, kets, terms, paths = _hubbard_setup((2, 3), (2, 2), 35)
    gterms = [(AG.DTensor.from_tensor(GP.operator_tensor(spec, operator_dense(kind, "Z2"))), sites)
              for kind, sites in W.hubbard_terms(spec)]
    D0 = [_dtensor(k) for k in kets]
    E0 = AG.expectation_ratio(spec, D0, gterms, paths, chi=6)
    g0 = torch.autograd.grad(E0, [x.data for x in D0])
    D1 = [_dtensor(k) for k in kets]
    E1 = AG.expectation_ratio(spec, D1, gterms, paths, chi=6, checkpoint=ck)
    assert float(E1.detach()) == float(E0.detach())
    g1 = torch.autograd.grad(E1, [x.data for x in D1])
    for s in range(len(kets)):
        a, b = g0[s].double().cpu().numpy(), g1[s].double().cpu().numpy()
        assert np.abs(a - b).max(initial=0) <= 1e-12 * max(1e-300, np.abs(a).max(initial=0)), s


def test_checkpointed_network_gradient_keeps_only_segment_inputs(P):
    # a compressed norm network: with one checkpoint per step the graph holds
    # the segment functions only, and the gradient equals the stored one
    from paper_2410_02215_amd import autograd as AG
    from tests.test_oracle_adjoint import _hubbard_setup
    spec, kets, terms, paths = _hubbard_setup((2, 3), (2, 2), 36)
    outs = []
    for ck in (None, 1):
        D = [_dtensor(k) for k in kets]
        t, b, p = AG.norm_tensors(spec, D)
        F, _, e2 = AG.contract(t, b, paths[None], 6, p, checkpoint=ck)
        v = F.data.sum()
        names = set()
        stack = [v.grad_fn]
        while stack:
            fn = stack.pop()
            if fn is None:
                continue
            names.add(type(fn).__name__)
            stack.extend(f for f, _ in fn.next_functions)
        outs.append((float(v.detach()), e2, torch.autograd.grad(v, [x.data for x in D]), names))
    (v0, e0, g0, n0), (v1, e1, g1, n1) = outs
    assert (v1, e1) == (v0, e0)
    assert any("_Dot" in n for n in n0) and any("_Compress" in n for n in n0)
    assert not any("_Dot" in n or "_Compress" in n for n in n1) and any("_Segment" in n for n in n1)
    for a, b in zip(g0, g1):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        assert np.abs(a - b).max(initial=0) <= 1e-12 * max(1e-300, np.abs(a).max(initial=0))


def test_differentiation_workload_hop_gradient_at_chi32(P):
    # the 6 x 6 differentiation lattice at its chi = 32: value and gradient of
    # <psi|h_(13,14)|psi>, whose compressions include bond sectors of 256
    # (block Jacobi eigenpairs in the compression adjoint), against the
    # oracle's values in tests/golden/values.json; recomputation segments of
    # one lattice layer
    import json
    import os
    from paper_2410_02215_amd import peps as GP
    from synth import workloads as W
    from synth.operators import operator_dense
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    gold = json.load(open(os.path.join(root, "tests", "golden", "values.json")))["c5_hop_grad"]
    cfg = W.c5()
    spec = cfg["spec"]
    sites = tuple(gold["op_sites"])
    kets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    op = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    net = GP.norm_network(spec, kets, op=op, op_sites=sites)
    path = W.norm_layer_path(spec, cfg["lx"], cfg["ly"], sites)
    m, e, g = net.contract_grad(path, chi=gold["chi"], checkpoint=cfg["ly"])
    ref = gold["mantissa"] * 2.0 ** gold["exp2"]
    verr = abs(m * 2.0 ** e - ref) / abs(ref)
    gerr = perr = 0.0
    for t, (g2, pr) in enumerate(zip(gold["grad_sq"], gold["grad_probe"])):
        x = g[t].data().cpu().numpy() * 2.0 ** e
        r = np.random.default_rng(7000 + t).standard_normal(x.size)
        gerr = max(gerr, abs(float(x @ x) - g2) / g2)
        # probe error against the Cauchy-Schwarz scale |g| |r|
        perr = max(perr, abs(float(x @ r) - pr) / np.sqrt(g2 * x.size))
    print("[c5 chi32] value rel err %.3g, |g|^2 rel err %.3g, probe err %.3g" % (verr, gerr, perr))
    # measured: about 4e-13, 1e-12 and 2e-13
    assert verr <= 1e-10
    assert gerr <= 1e-10
    assert perr <= 1e-10


def test_network_gradient_and_axpy_reject_unsupported_arguments(P):
    # FP32 tensors or GEMM forms, an open network and a negative checkpoint
    # are refused with an error code; axpy needs one structure
    rng = np.random.default_rng(36)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rand_tensor(rng, sym, [l(2, 2, 0), l(3, 1, 1)], total=(0,))
    B = rand_tensor(rng, sym, [l(3, 1, 0), l(2, 2, 1)], total=(0,))
    closed = P.Network([to_gpu(A), to_gpu(B)], [(0, 0, 1, 1), (0, 1, 1, 0)], conv=P.LOCAL)
    with pytest.raises(P.FtnError) as e:
        closed.contract_grad([(0, 1)], chi=0, gemm=P.GEMM_F32)
    assert e.value.code == -6  # FTN_ENOTSUP
    with pytest.raises(P.FtnError) as e:
        closed.contract_grad([(0, 1)], chi=0, checkpoint=-1)
    assert e.value.code == -1  # FTN_EINVAL
    opened = P.Network([to_gpu(A), to_gpu(B)], [(0, 1, 1, 0)], conv=P.LOCAL)
    with pytest.raises(P.FtnError) as e:
        opened.contract_grad([(0, 1)], chi=0)
    assert e.value.code == -6
    with pytest.raises(P.FtnError) as e:
        P.ftn.axpy(1.0, to_gpu(A), to_gpu(B))
    assert e.value.code == -1
    # the exact gradient of the closed pair is the other tensor, arranged
    m, ex, g = closed.contract_grad([(0, 1)], chi=0)
    assert len(g) == 2 and m != 0.0
