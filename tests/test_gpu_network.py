"""GPU parity of bond compression and network contraction (via the C ABI).

Exact contractions agree with the oracle to FP64 rounding (1e-12 relative).
Compression: the compressed pair's contraction F(A'B') is gauge invariant
and is compared with the oracle's; the library factors Gram matrices (so a
direction with singular value s is resolved to ~eps * s_max^2 / s), which
bounds the agreement of truncated results at 1e-9 relative on these
inputs. Integer results (kept sector dims) must be identical.
"""

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from oracle import physics as OP
from oracle.linalg import compress_bond as o_compress
from oracle.network import Network as ONet, contract_network as o_contract, network_value
from oracle.ops import ftensordot, ftranspose
from synth import workloads as W
from synth.operators import operator_dense
from tests.helpers import rand_leg, partner, rand_tensor, random_network, random_ssa_path
from tests.gpu_helpers import to_gpu, from_gpu, assert_same_structure

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2410_02215_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    P.load_library()
    return P


def _val(m, e):
    return m * 2.0 ** e


@pytest.mark.parametrize("conv", ["local", "global"])
def test_c1_exact_norm(P, conv):
    from paper_2410_02215_amd import peps as GP
    cfg = W.c1()
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"], std=cfg["std"])
    onet = OP.norm_network(spec, OP.ket_tensors(spec, vals), conv=conv)
    path = W.norm_path(spec, seed=0)
    ref = _val(*network_value(onet, path))
    gnet = GP.norm_network(spec, GP.ket_tensors(spec, vals), conv=P.LOCAL if conv == "local" else P.GLOBAL)
    m, e, st = gnet.contract(path)
    assert abs(_val(m, e) - ref) <= 1e-12 * abs(ref)
    # a second, different path gives the same value (order invariance)
    p2 = W.norm_path(spec, seed=5, pair_layers=False)
    m2, e2, _ = gnet.contract(p2)
    assert abs(_val(m2, e2) - ref) <= 1e-12 * abs(ref)


def _flat_perm(labels, order, ndims):
    flat = [(t, l) for t in order for l in range(ndims[t])]
    rank = {x: k for k, x in enumerate(flat)}
    return sorted(range(len(labels)), key=lambda k: rank[tuple(labels[k])])


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1])
@pytest.mark.parametrize("seed", range(4))
def test_random_networks_with_odd_tensors(P, sym, conv, seed):
    rng = np.random.default_rng(700 + seed)
    nt = int(rng.integers(2, 6))
    tensors, bonds = random_network(rng, sym, nt, nt + 1, n_open=int(rng.integers(0, 3)), odd_frac=0.5)
    pos = list(rng.permutation(nt))
    order = sorted(range(nt), key=lambda t: pos[t])
    onet = ONet(tensors, bonds, conv="global", positions=pos)
    path = random_ssa_path(rng, tensors, bonds)
    T, labs, e, _ = o_contract(onet, path)
    perm = _flat_perm([(l[1], l[2]) for l in labs], order, {t: x.ndim for t, x in tensors.items()})
    ref = ftranspose(T, perm).to_dense() * 2.0 ** e
    g = [to_gpu(tensors[t]) for t in range(nt)]
    gnet = P.Network(g, bonds, conv=P.GLOBAL if conv == "global" else P.LOCAL, positions=pos)
    if conv == "local":
        # the same network in local form: the oracle's translation defines it
        from oracle.network import to_local
        loc = to_local(onet)
        g = [to_gpu(loc.tensors[t]) for t in range(nt)]
        gnet = P.Network(g, bonds, conv=P.LOCAL, positions=pos)
    if T.ndim == 0:
        m, ge, _ = gnet.contract(path)
        assert abs(_val(m, ge) - float(ref)) <= 1e-12 * max(1.0, abs(float(ref)))
    else:
        G, ge, src, _ = gnet.contract(path, open_legs=True)
        gp = _flat_perm(src, order, {t: x.ndim for t, x in tensors.items()})
        Gt = P.ftranspose(G, gp)
        got = Gt.to_dense().cpu().numpy() * 2.0 ** ge
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", [S.Z2, S.U1, S.U1U1])
def test_compress_bond_matches_oracle(P, sym, conv):
    rng = np.random.default_rng(800)
    for trial in range(5):
        bond = rand_leg(rng, sym, maxd=6)
        la = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        lb = [rand_leg(rng, sym, maxd=3) for _ in range(2)]
        pa, pb = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        A = rand_tensor(rng, sym, la[:pa] + [bond] + la[pa:], total=S.zero(sym))
        B = rand_tensor(rng, sym, lb[:pb] + [partner(bond)] + lb[pb:], total=S.zero(sym))
        chi = int(rng.integers(2, 8))
        A2, B2, info = o_compress(A, B, pa, pb, chi, conv=conv, cutoff=1e-12)
        ref = ftensordot(A2, B2, [pa], [pb], conv).to_dense()
        cv = P.LOCAL if conv == "local" else P.GLOBAL
        GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), pa, pb, chi, 1e-12, cv)
        assert GA.legs()[pa][1] == list(A2.legs[pa].dims)       # kept dims, bit-exact
        GC = P.ftensordot(GA, GB, [pa], [pb], conv=cv)
        got = GC.to_dense().cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * max(1.0, np.abs(ref).max()))
        kept = sorted(np.concatenate([v.numpy() for v in info["svals"].values()]), reverse=True)
        np.testing.assert_allclose(ginfo["svals"], kept, rtol=1e-9)


@pytest.mark.parametrize("chi,kept", [(100, {(0,): 7, (1,): 6}), (10, {(0,): 6, (1,): 4})])
def test_compress_bond_resolves_a_graded_spectrum(P, chi, kept):
    # bond matrices with singular values from 1 down to 1e-15 per Z2 sector:
    # with cutoff 1e-12 the kept dims are fixed by values down to 4e-11, so
    # the library must resolve singular values far below the ~1e-8 of a Gram
    # matrix; kept dims bit-exact, kept values to 1e-14 of the largest
    rng = np.random.default_rng(830)
    sym = S.Z2
    from oracle.tensor import make_leg, FTensor
    sig = {0: [1.0, 3e-2, 1e-3, 3e-5, 1e-6, 3e-8, 1e-9, 1e-14],
           1: [0.5, 2e-3, 4e-6, 8e-9, 2e-10, 4e-11, 3e-13, 1e-15]}
    la = make_leg(sym, [(0,), (1,)], [20, 20], 0)
    bond = make_leg(sym, [(0,), (1,)], [8, 8], 1)
    lb = make_leg(sym, [(0,), (1,)], [12, 12], 1)
    A = FTensor.zeros(sym, [la, bond], (0,))
    B = FTensor.zeros(sym, [partner(bond), lb], (0,))
    for q in (0, 1):
        ua = np.linalg.qr(rng.standard_normal((20, 8)))[0]
        va = np.linalg.qr(rng.standard_normal((8, 8)))[0]
        wb = np.linalg.qr(rng.standard_normal((12, 8)))[0].T
        A.blocks[(q, q)] = torch.from_numpy(ua @ np.diag(sig[q]) @ va.T)
        B.blocks[(q, q)] = torch.from_numpy(wb.copy())
    A2, B2, info = o_compress(A, B, 1, 0, chi, conv="local", cutoff=1e-12)
    assert {q: len(v) for q, v in info["svals"].items()} == kept
    GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi, 1e-12, P.LOCAL)
    assert GA.legs()[1][1] == [kept[(0,)], kept[(1,)]]
    ref_sv = sorted(np.concatenate([v.numpy() for v in info["svals"].values()]), reverse=True)
    np.testing.assert_allclose(ginfo["svals"], ref_sv, rtol=0, atol=1e-14)
    ref = ftensordot(A2, B2, [1], [0], "local").to_dense()
    got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("sym", [S.Z2, S.U1])
def test_compress_bond_odd_tensors(P, sym):
    # network bodies of odd tensors are compressed without dummy legs
    rng = np.random.default_rng(802)
    for trial, (ta, tb) in enumerate([((1,), (1,)), ((1,), (0,)), ((0,), (1,)), ((1,), (1,))]):
        bond = rand_leg(rng, sym, maxd=6)
        A = rand_tensor(rng, sym, [rand_leg(rng, sym, maxd=3), bond, rand_leg(rng, sym, maxd=3)], total=ta)
        B = rand_tensor(rng, sym, [partner(bond), rand_leg(rng, sym, maxd=3)], total=tb)
        chi = int(rng.integers(2, 8))
        A2, B2, info = o_compress(A, B, 1, 0, chi, conv="local", cutoff=1e-12)
        ref = ftensordot(A2, B2, [1], [0], "local").to_dense()
        GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi, 1e-12, P.LOCAL)
        assert GA.legs()[1][1] == list(A2.legs[1].dims)
        got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("seed", range(4))
def test_random_networks_with_odd_tensors_compressed(P, seed):
    # odd tensors, parallel bonds fused and compressed: the sign bookkeeping
    # of the dummies must agree with the oracle's materialised dummy legs
    # (Z2: random U(1) totals almost never close to a nonzero value)
    sym = S.Z2
    rng = np.random.default_rng(710 + seed)
    chi = 3
    while True:
        nt = int(rng.integers(4, 7))
        tensors, bonds = random_network(rng, sym, nt, nt + 3, odd_frac=0.5, maxd=3)
        if sum(tensors[t].parity for t in tensors) % 2:
            continue
        pos = [int(x) for x in rng.permutation(nt)]
        path = random_ssa_path(rng, tensors, bonds)
        onet = ONet(tensors, bonds, conv="local", positions=pos)
        T, labs, e, infos = o_contract(onet, path, chi=chi)
        ref = (float(T.blocks[()]) if () in T.blocks else 0.0) * 2.0 ** e
        if ref != 0.0 and infos and sum(1 for t in tensors.values() if t.parity) >= 2:
            break
    gnet = P.Network([to_gpu(tensors[t]) for t in range(nt)], bonds, conv=P.LOCAL, positions=pos)
    m, ge, _ = gnet.contract(path, chi=chi)
    assert abs(_val(m, ge) - ref) <= 1e-9 * max(abs(ref), 1e-300), (m, ge, ref)


def test_compress_large_sector_subspace_iteration(P):
    # bond sectors above 128 exercise the subspace-iteration SVD path
    rng = np.random.default_rng(801)
    sym = S.Z2
    from oracle.tensor import make_leg
    bond = make_leg(sym, [(0,), (1,)], [150, 140], 1)
    A = rand_tensor(rng, sym, [make_leg(sym, [(0,), (1,)], [200, 180], 0), bond], total=(0,))
    B = rand_tensor(rng, sym, [partner(bond), make_leg(sym, [(0,), (1,)], [170, 190], 1)], total=(0,))
    chi = 64
    A2, B2, info = o_compress(A, B, 1, 0, chi)
    ref = ftensordot(A2, B2, [1], [0]).to_dense()
    GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi)
    assert GA.legs()[1][1] == list(A2.legs[1].dims)
    got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("n_sites,chi", [(8, 16), (12, 24)])
def test_approximate_norm_and_hopping_small_rrg(P, n_sites, chi):
    from paper_2410_02215_amd import peps as GP
    cfg = W.c2(n_sites=n_sites, chi=chi)
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"])
    okets = OP.ket_tensors(spec, vals)
    path = W.norm_path(spec, chi=chi, seed=1)
    ref = _val(*network_value(OP.norm_network(spec, okets, conv="local"), path, chi=chi))
    gk = GP.ket_tensors(spec, vals)
    m, e, st = GP.norm_network(spec, gk).contract(path, chi=chi)
    assert abs(_val(m, e) - ref) <= 1e-9 * abs(ref)
    assert st["compressions"] > 0
    # hopping term on the first edge
    u, v = cfg["op_sites"]
    G = OP.operator_tensor(OP.two_site_local("hop"), okets[0].legs[0], S.Z2)
    p2 = W.norm_path(spec, chi=chi, seed=1, op_sites=(u, v))
    oref = _val(*network_value(OP.norm_network(spec, okets, op=G, op_sites=(u, v), conv="local"), p2, chi=chi))
    gop = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    m2, e2, _ = GP.norm_network(spec, gk, op=gop, op_sites=(u, v)).contract(p2, chi=chi)
    # the hopping term is measured against its own magnitude
    assert abs(_val(m2, e2) - oref) <= 1e-9 * abs(oref), (_val(m2, e2), oref)


def test_compress_rank_deficient_subspace_iteration(P):
    # both sides have rank > 128 but their product has rank <= 2 x 60: the
    # subspace iteration meets exactly dependent directions
    rng = np.random.default_rng(802)
    sym = S.Z2
    from oracle.tensor import make_leg, FTensor
    bond = make_leg(sym, [(0,), (1,)], [300, 300], 1)
    ra = make_leg(sym, [(0,), (1,)], [200, 200], 0)
    rb = make_leg(sym, [(0,), (1,)], [200, 200], 1)
    Ad = np.zeros((400, 600))
    Bd = np.zeros((600, 400))
    for s in range(2):
        r0, b0 = 200 * s, 300 * s
        Ad[r0:r0 + 200, b0:b0 + 180] = rng.standard_normal((200, 180))
        Bd[b0 + 120:b0 + 300, r0:r0 + 200] = rng.standard_normal((180, 200))
    A = FTensor.from_dense(sym, [ra, bond], (0,), Ad)
    B = FTensor.from_dense(sym, [partner(bond), rb], (0,), Bd)
    chi = 100
    A2, B2, info = o_compress(A, B, 1, 0, chi, cutoff=1e-6)
    ref = ftensordot(A2, B2, [1], [0]).to_dense()
    GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi, 1e-6)
    assert GA.legs()[1][1] == list(A2.legs[1].dims)
    got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("dims", [(100, 300), (128, 129), (60, 40)])
def test_compress_mixed_sector_sizes(P, dims):
    # one bond sector small enough for the direct eigensolver, one that
    # needs subspace iteration (or both small), with decaying spectra
    rng = np.random.default_rng(803 + dims[0])
    sym = S.Z2
    from oracle.tensor import make_leg, FTensor
    bond = make_leg(sym, [(0,), (1,)], list(dims), 1)
    ra = make_leg(sym, [(0,), (1,)], [150, 170], 0)
    rb = make_leg(sym, [(0,), (1,)], [160, 140], 1)
    A = FTensor.zeros(sym, [ra, bond], (0,))
    B = FTensor.zeros(sym, [partner(bond), rb], (0,))
    for q in range(2):
        d = dims[q]
        m, n = ra.dims[q], rb.dims[q]
        A.blocks[(q, q)] = torch.from_numpy(rng.standard_normal((m, d)) * np.logspace(0, -5, d)[None, :])
        B.blocks[(q, q)] = torch.from_numpy(np.logspace(0, -3, d)[:, None] * rng.standard_normal((d, n)))
    chi = 90
    A2, B2, info = o_compress(A, B, 1, 0, chi, cutoff=1e-6)
    ref = ftensordot(A2, B2, [1], [0]).to_dense()
    GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi, 1e-6)
    assert GA.legs()[1][1] == list(A2.legs[1].dims)
    got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_compress_many_sectors_repeat_is_bit_exact(P):
    # a U(1) bond of 12 sectors: the factorisation kernels take their job
    # tables from an upload (more than eight sectors, the most the kernel
    # arguments carry); a second identical call takes every grouped-product
    # plan from the plan cache and reproduces the first bit for bit
    from oracle.tensor import make_leg
    rng = np.random.default_rng(907)
    sym = S.U1
    qs = [(q,) for q in range(-5, 7)]
    bond = make_leg(sym, qs, [int(x) for x in rng.integers(3, 14, len(qs))], 1)
    ra = make_leg(sym, qs, [int(x) for x in rng.integers(10, 40, len(qs))], 0)
    rb = make_leg(sym, qs, [int(x) for x in rng.integers(10, 40, len(qs))], 1)
    A = rand_tensor(rng, sym, [ra, bond], total=(0,))
    B = rand_tensor(rng, sym, [partner(bond), rb], total=(0,))
    chi = 40
    A2, B2, info = o_compress(A, B, 1, 0, chi, cutoff=1e-12)
    ref = ftensordot(A2, B2, [1], [0]).to_dense()
    ga, gb = to_gpu(A), to_gpu(B)
    outs = []
    for _ in range(2):
        GA, GB, _ = P.compress_bond(ga, gb, 1, 0, chi, 1e-12)
        assert GA.legs()[1][1] == list(A2.legs[1].dims)
        outs.append(P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy())
    np.testing.assert_allclose(outs[0], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("case", [
    # the thin route needs A~ sectors of at least 2^22 entries (M d); the
    # small shapes beside them take the Gram route with the same structure
    ((90, 70), (50000, 60000), (8, 5), 20),     # d <= 128, thin B side, nothing truncated
    ((90, 70), (300, 260), (8, 5), 20),         # the same shape, small: Gram route
    ((120, 100), (36000, 42000), (60, 40), 30),  # d <= 128, thin B side, truncated
    ((120, 100), (900, 700), (60, 40), 30),     # small: Gram route
    ((300, 200), (700, 500), (100, 128), 60),   # d > 128 (the Gram route) beside the same shapes
    ((80, 60), (53000, 70000), (16, 12), 10),   # thin, with B~ of rank below N
    # the Gram of Y = A~ B~ (N <= 32 columns, ragged long sides) takes the
    # tall-skinny A^T B kernel; N = 1
    ((100, 80), (42001, 53000), (24, 9), 25),
    ((128, 64), (33000, 65601), (32, 1), 20),
    # Y = A~ B~ with N <= 16 takes the streaming tall kernel
    ((64, 48), (66000, 88000), (16, 7), 20),
])
def test_compress_thin_b_side_matches_oracle(P, case):
    # sectors whose B side is thin (N <= d, N <= 128) and A~ tall (M > d):
    # spectrum from the QR of Y = A~ B~, B projector through a left inverse
    # of B~; kept dims bit-exact and the compressed product against the oracle
    (d0, d1), (m0, m1), (n0, n1), chi = case
    rng = np.random.default_rng(811 + d0)
    sym = S.Z2
    from oracle.tensor import make_leg, FTensor
    bond = make_leg(sym, [(0,), (1,)], [d0, d1], 1)
    ra = make_leg(sym, [(0,), (1,)], [m0, m1], 0)
    rb = make_leg(sym, [(0,), (1,)], [n0, n1], 1)
    A = FTensor.zeros(sym, [ra, bond], (0,))
    B = FTensor.zeros(sym, [partner(bond), rb], (0,))
    for q, (m, d, n) in enumerate(((m0, d0, n0), (m1, d1, n1))):
        A.blocks[(q, q)] = torch.from_numpy(rng.standard_normal((m, d)))
        Bq = rng.standard_normal((d, n)) * np.logspace(0, -2, n)[None, :]
        if chi == 10:  # two dependent columns of B~
            Bq[:, -1] = Bq[:, 0] - 2.0 * Bq[:, 1]
        B.blocks[(q, q)] = torch.from_numpy(Bq)
    A2, B2, info = o_compress(A, B, 1, 0, chi, cutoff=1e-12)
    ref = ftensordot(A2, B2, [1], [0]).to_dense()
    GA, GB, ginfo = P.compress_bond(to_gpu(A), to_gpu(B), 1, 0, chi, 1e-12)
    assert GA.legs()[1][1] == list(A2.legs[1].dims)
    got = P.ftensordot(GA, GB, [1], [0]).to_dense().cpu().numpy()
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_concurrent_contractions_on_two_streams(P):
    # two independent approximate contractions issued from two host threads on
    # two streams give exactly the results of running them one after another
    import threading
    from paper_2410_02215_amd import peps as GP
    cfg = W.c2(n_sites=12, chi=24)
    spec = cfg["spec"]
    kets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    op = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    nets = [GP.norm_network(spec, kets), GP.norm_network(spec, kets, op=op, op_sites=cfg["op_sites"])]
    paths = [W.norm_path(spec, chi=24, seed=1), W.norm_path(spec, chi=24, seed=1, op_sites=cfg["op_sites"])]
    serial = [nets[k].contract(paths[k], chi=24)[:2] for k in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]

    def run(k):
        with torch.cuda.stream(streams[k]):
            for _ in range(3):
                out[k] = nets[k].contract(paths[k], chi=24)[:2]

    th = threading.Thread(target=run, args=(1,))
    th.start()
    run(0)
    th.join()
    torch.cuda.synchronize()
    assert out == serial


def test_c2_repeated_and_concurrent_contractions_are_bitwise_identical(P):
    # Repeating the 40-site contractions, one after the other and then the
    # norm and the hopping term at the same time on two streams from two host
    # threads, must reproduce the first results bit for bit: no kernel may
    # depend on wave timing, and no buffer may be reused by one stream while
    # another still reads it.
    import json, os, threading
    from paper_2410_02215_amd import peps as GP
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    paths = json.load(open(os.path.join(root, "synth", "data", "paths.json")))
    cfg = W.c2()
    spec = cfg["spec"]
    kets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    op = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    nets = [GP.norm_network(spec, kets), GP.norm_network(spec, kets, op=op, op_sites=cfg["op_sites"])]
    pth = [paths["c2_norm"]["path"], paths["c2_hop"]["path"]]
    torch.cuda.synchronize()

    def one(k):
        m, e, _ = nets[k].contract(pth[k], chi=cfg["chi"])
        return (m, e)

    ref = [one(0), one(1)]
    for _ in range(3):
        assert [one(0), one(1)] == ref
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for _ in range(4):
        out = [None, None]

        def run(k):
            with torch.cuda.stream(streams[k]):
                out[k] = one(k)

        th = threading.Thread(target=run, args=(1,))
        th.start()
        run(0)
        th.join()
        torch.cuda.synchronize()
        assert out == ref


def test_c2_full_size_norm_and_hopping(P):
    # the full 40-site workload against the stored oracle values
    import json, os
    from paper_2410_02215_amd import peps as GP
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    gold = json.load(open(os.path.join(root, "tests", "golden", "values.json")))
    paths = json.load(open(os.path.join(root, "synth", "data", "paths.json")))
    cfg = W.c2()
    spec = cfg["spec"]
    kets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    m, e, st = GP.norm_network(spec, kets).contract(paths["c2_norm"]["path"], chi=cfg["chi"])
    ref = gold["c2_norm"]["mantissa"] * 2.0 ** gold["c2_norm"]["exp2"]
    print("c2 norm gpu %.15g ref %.15g rel %.3g near_ties %d" % (_val(m, e), ref, abs(_val(m, e) / ref - 1),
                                                                   st["near_ties"]))
    # measured 1.8e-13 (norm) and 5.1e-13 (hopping term)
    assert abs(_val(m, e) - ref) <= 1e-10 * abs(ref)
    op = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    m2, e2, _ = GP.norm_network(spec, kets, op=op, op_sites=cfg["op_sites"]).contract(paths["c2_hop"]["path"],
                                                                                    chi=cfg["chi"])
    ref2 = gold["c2_hop"]["mantissa"] * 2.0 ** gold["c2_hop"]["exp2"]
    print("c2 hop gpu %.15g ref %.15g rel %.3g" % (_val(m2, e2), ref2, abs(_val(m2, e2) / ref2 - 1)))
    # the hopping term is measured against its own magnitude
    assert abs(_val(m2, e2) - ref2) <= 1e-10 * abs(ref2)


def test_precision_forms_on_a_u1u1_diamond_cluster(P):
    # the precision workload's structure (U(1)xU(1) diamond lattice, bond
    # (0,0):4 and four charged sectors of 1) on a 2x2x1-cell cluster: the
    # FP64 path against the oracle, then FP32 tensors with FP32 and split-BF16
    # block GEMMs (compression in FP64) against the same oracle value
    from paper_2410_02215_amd import peps as GP
    cfg = W.c3(cells=(2, 2, 1), chi=16)
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"])
    okets = OP.ket_tensors(spec, vals)
    path = W.norm_path(spec, chi=16, seed=1)
    ref = _val(*network_value(OP.norm_network(spec, okets, conv="local"), path, chi=16))
    gk = GP.ket_tensors(spec, vals)
    m, e, st = GP.norm_network(spec, gk).contract(path, chi=16)
    assert st["compressions"] > 0
    err64 = abs(_val(m, e) - ref) / abs(ref)
    assert err64 <= 1e-9, err64
    gk32 = []
    for k in gk:
        inf = k.info()
        gk32.append(P.Tensor.create(inf["sym"], k.legs(), inf["total"], P.F32, data=k.data().float()))
    # the FP32 tensors hold the inputs rounded to nearest: the oracle on the
    # same rounded values isolates the error of the FP32 arithmetic; the error
    # against the unrounded oracle value is reported beside it
    vals32 = [v.astype(np.float32).astype(np.float64) for v in vals]
    ref32 = _val(*network_value(OP.norm_network(spec, OP.ket_tensors(spec, vals32), conv="local"), path, chi=16))
    errs, errs_in = {}, {}
    for name, gemm, tol in (("f32", P.GEMM_F32, 1e-6), ("bf16x3", P.GEMM_BF16X3, 1e-4)):
        m3, e3, _ = GP.norm_network(spec, gk32).contract(path, chi=16, gemm=gemm)
        errs[name] = abs(_val(m3, e3) - ref32) / abs(ref32)
        errs_in[name] = abs(_val(m3, e3) - ref) / abs(ref)
        assert errs[name] <= tol, (name, errs[name])
    print("relative error vs the FP64 oracle on the rounded inputs: fp64 %.3g, fp32 %.3g, bf16x3 %.3g; "
          "vs the unrounded inputs: fp32 %.3g, bf16x3 %.3g"
          % (err64, errs["f32"], errs["bf16x3"], errs_in["f32"], errs_in["bf16x3"]))


def test_precision_workload_on_a_16_site_cluster(P):
    # the precision workload's structure (U(1)xU(1) diamond cluster, bond
    # (0,0):4 plus four charged sectors of 1, compression as early as
    # possible) on 2 x 2 x 2 cells (16 sites) at chi = 32, the largest cluster
    # the oracle contracts in minutes (tests/golden/make_golden.py): FP64 path,
    # then FP32 tensors with FP32 and split-BF16 block GEMMs (compression in
    # FP64), each against the FP64 oracle value
    import json, os, time
    from paper_2410_02215_amd import peps as GP
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    gold = json.load(open(os.path.join(root, "tests", "golden", "values.json")))["c3_222_norm"]
    ref = gold["mantissa"] * 2.0 ** gold["exp2"]
    cfg = W.c3(cells=(2, 2, 2), chi=32)
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"])
    path = W.norm_path(spec, chi=32, seed=0)
    gk = GP.ket_tensors(spec, vals)
    torch.cuda.synchronize()
    t0 = time.time()
    m, e, st = GP.norm_network(spec, gk).contract(path, chi=32)
    t64 = time.time() - t0
    assert st["compressions"] > 0
    err64 = abs(_val(m, e) - ref) / abs(ref)
    gk32 = []
    for k in gk:
        inf = k.info()
        gk32.append(P.Tensor.create(inf["sym"], k.legs(), inf["total"], P.F32, data=k.data().float()))
    errs, secs = {}, {}
    for name, gemm in (("f32", P.GEMM_F32), ("bf16x3", P.GEMM_BF16X3)):
        torch.cuda.synchronize()
        t0 = time.time()
        m3, e3, _ = GP.norm_network(spec, gk32).contract(path, chi=32, gemm=gemm)
        secs[name] = time.time() - t0
        errs[name] = abs(_val(m3, e3) - ref) / abs(ref)
    print("16-site U1xU1 cluster chi 32: relative error vs the FP64 oracle fp64 %.3g (%.2f s), fp32 %.3g (%.2f s), "
          "bf16x3 %.3g (%.2f s); %d compressions" % (err64, t64, errs["f32"], secs["f32"], errs["bf16x3"],
                                                     secs["bf16x3"], st["compressions"]))
    assert err64 <= 1e-10, err64
    # against the FP64 value of the unrounded inputs, so the FP32 input
    # rounding is included (measured 9.4e-7; the arithmetic alone is held to
    # 1e-6 on rounded inputs in test_precision_forms_on_a_u1u1_diamond_cluster)
    assert errs["f32"] <= 2e-6, errs
    assert errs["bf16x3"] <= 2e-4, errs
