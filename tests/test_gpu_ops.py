"""GPU parity of the elementary operations against the oracle (via the C ABI).

Integer work (block keys, offsets) and pure sign-carrying copies
(transposition, arrow reversal, fusion, dense gather) must be bit-exact.
Contractions in FP64 agree with the oracle up to summation order: the
tolerance is 64 * eps * sum_k |a_ik||b_kj| per entry (a forward error bound
of a length-k dot product), checked as a relative max error of 1e-12 on
these O(1) random inputs.
"""

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from oracle.ops import ftranspose, ftensordot, flip_dual, fuse
from oracle.tensor import FTensor, make_leg
from tests.helpers import rand_leg, partner, rand_tensor
from tests.gpu_helpers import to_gpu, from_gpu, assert_same_structure, flat_blocks, rounded_f32

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


@pytest.mark.parametrize("sym", SYMS)
def test_create_structure_and_gather_bit_exact(P, sym):
    rng = np.random.default_rng(1)
    for trial in range(8):
        n = int(rng.integers(0, 6))
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        G = to_gpu(T)
        assert_same_structure(T, G)
        np.testing.assert_array_equal(_data(G), flat_blocks(T))
        np.testing.assert_array_equal(G.to_dense().cpu().numpy(), T.to_dense())


def test_many_sectors_large_enumeration(P):
    # U(1) legs with many sectors: enumeration over tens of thousands of keys
    rng = np.random.default_rng(2)
    legs = [make_leg(S.U1, [(q,) for q in range(-4, 5)], [1] * 9, int(rng.integers(0, 2)))
            for _ in range(6)]
    T = FTensor.zeros(S.U1, legs, (1,))
    G = P.Tensor.create(1, [([(q[0], 0) for q in l.charges], list(l.dims), l.dual) for l in legs], (1, 0))
    assert_same_structure(T, G)


@pytest.mark.parametrize("sym", SYMS)
def test_ftranspose_bit_exact(P, sym):
    rng = np.random.default_rng(3)
    for trial in range(10):
        n = int(rng.integers(1, 7))
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        perm = list(rng.permutation(n))
        ref = ftranspose(T, perm)
        G = P.ftranspose(to_gpu(T), perm)
        assert_same_structure(ref, G)
        np.testing.assert_array_equal(_data(G), flat_blocks(ref))


@pytest.mark.parametrize("sym", SYMS)
def test_flip_dual_bit_exact(P, sym):
    rng = np.random.default_rng(4)
    for trial in range(6):
        n = int(rng.integers(1, 5))
        legs = [rand_leg(rng, sym, maxd=3) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        leg = int(rng.integers(0, n))
        for ws, ref in ((-1, flip_dual(T, leg)), (0, flip_dual(T, leg, with_sign=False)),
                        (1, flip_dual(T, leg, with_sign=True))):
            G = P.flip_dual(to_gpu(T), leg, ws)
            assert_same_structure(ref, G)
            np.testing.assert_array_equal(_data(G), flat_blocks(ref))


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", SYMS)
def test_fuse_bit_exact(P, sym, conv):
    rng = np.random.default_rng(5)
    for trial in range(6):
        n = int(rng.integers(2, 6))
        legs = [rand_leg(rng, sym, maxd=2) for _ in range(n)]
        T = rand_tensor(rng, sym, legs)
        m = int(rng.integers(2, n + 1))
        gl = [int(x) for x in rng.permutation(n)[:m]]
        rev = int(rng.integers(0, 2))
        ref, _ = fuse(T, gl, conv=conv, rev=rev)
        G = P.fuse(to_gpu(T), gl, conv=P.LOCAL if conv == "local" else P.GLOBAL, rev=rev)
        assert_same_structure(ref, G)
        np.testing.assert_array_equal(_data(G), flat_blocks(ref))


def _rand_pair(rng, sym, k, nfa, nfb, maxd):
    bond = [rand_leg(rng, sym, maxd=maxd) for _ in range(k)]
    fa = [rand_leg(rng, sym, maxd=maxd) for _ in range(nfa)]
    fb = [rand_leg(rng, sym, maxd=maxd) for _ in range(nfb)]
    A_legs = fa + bond
    B_legs = [partner(b) for b in bond] + fb
    pa = list(rng.permutation(len(A_legs)))
    pb = list(rng.permutation(len(B_legs)))
    A = rand_tensor(rng, sym, [A_legs[p] for p in pa])
    B = rand_tensor(rng, sym, [B_legs[p] for p in pb])
    ax_a = [pa.index(nfa + t) for t in range(k)]
    ax_b = [pb.index(t) for t in range(k)]
    return A, B, ax_a, ax_b


@pytest.mark.parametrize("conv", ["local", "global"])
@pytest.mark.parametrize("sym", SYMS)
def test_ftensordot_fp64(P, sym, conv):
    rng = np.random.default_rng(6)
    for trial in range(8):
        k = int(rng.integers(0, 4))
        A, B, ax_a, ax_b = _rand_pair(rng, sym, k, int(rng.integers(0, 4)), int(rng.integers(0, 4)), 3)
        ref = ftensordot(A, B, ax_a, ax_b, conv=conv)
        G = P.ftensordot(to_gpu(A), to_gpu(B), ax_a, ax_b,
                         conv=P.LOCAL if conv == "local" else P.GLOBAL)
        assert_same_structure(ref, G)
        r = flat_blocks(ref)
        np.testing.assert_allclose(_data(G), r, rtol=0, atol=1e-12 * max(1.0, np.abs(r).max(initial=0)))


def test_ftensordot_tiles_and_ragged_tails(P):
    # large sectors: several 64 x 64 tiles per group plus ragged edges
    rng = np.random.default_rng(7)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rand_tensor(rng, sym, [l(37, 41, 0), l(70, 9, 1), l(13, 30, 0)], total=(0,))
    B = rand_tensor(rng, sym, [l(13, 30, 1), l(150, 3, 0)], total=(1,))
    ref = ftensordot(A, B, [2], [0], conv="local")
    G = P.ftensordot(to_gpu(A), to_gpu(B), [2], [0])
    assert_same_structure(ref, G)
    r = flat_blocks(ref)
    np.testing.assert_allclose(_data(G), r, rtol=0, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("case", [
    # (A legs, B legs, contracted legs of A): tall fused A (M >= 4096), N <= 16
    # and K <= 256 take the streaming tall kernel; odd K reads A entry by
    # entry, K % 4 == 0 in pairs; ragged M; N of 1; several row combos
    (((5000, 4200, 0), (40, 37, 1)), ((40, 37, 0), (9, 16, 1)), [1]),
    (((4500, 6000, 0), (64, 128, 1)), ((64, 128, 0), (1, 12, 1)), [1]),
    (((70, 65, 0), (80, 75, 0), (128, 128, 1)), ((128, 128, 0), (5, 3, 1)), [2]),
    (((300, 257, 0), (16, 16, 0), (256, 252, 1)), ((256, 252, 0), (16, 15, 1)), [2]),
])
def test_ftensordot_tall_thin_products(P, case):
    la, lb, ax = case
    rng = np.random.default_rng(sum(d for l in la for d in l[:2]))
    sym = S.Z2
    A = rand_tensor(rng, sym, [make_leg(sym, [(0,), (1,)], [e, o], d) for e, o, d in la], total=(0,))
    B = rand_tensor(rng, sym, [make_leg(sym, [(0,), (1,)], [e, o], d) for e, o, d in lb], total=(0,))
    from paper_2410_02215_amd import ftn
    ref = ftensordot(A, B, ax, [0], conv="local")
    ga, gb = to_gpu(A), to_gpu(B)
    torch.cuda.synchronize()
    ftn.profile_collect()
    ftn.profile_enable(True)
    G = P.ftensordot(ga, gb, ax, [0])
    torch.cuda.synchronize()
    ftn.profile_enable(False)
    assert ftn.profile_collect()["k_gemm_f64_tall"][1] == 1
    assert_same_structure(ref, G)
    r = flat_blocks(ref)
    np.testing.assert_allclose(_data(G), r, rtol=0, atol=1e-12 * np.abs(r).max())


def _u1_leg(dims, dual, qs=(-1, 0, 1)):
    return make_leg(S.U1, [(q,) for q in qs[:len(dims)]], dims, dual)


@pytest.mark.parametrize("case", [
    # (sym, A legs, B legs, contracted legs of A and of B, A read in place)
    # A's legs in fused order, one contracted sector combination per charge
    # group and long row combinations: the product reads A's blocks in place
    ("z2", [(40, 24, 0), (33, 31, 0), (64, 64, 1)], [(64, 64, 0), (20, 12, 1)], [2], [0], True),
    ("z2g", [(40, 24, 0), (33, 31, 0), (64, 64, 1)], [(64, 64, 0), (20, 12, 1)], [2], [0], True),
    # two contracted legs, the second with a single sector
    ("u1", [((30, 50, 40), 0), ((60, 70), 0), ((64, 48), 1), ((3,), 1)],
     [((64, 48), 0), ((3,), 0), ((5, 6, 7), 1)], [2, 3], [0, 1], True),
    # the contracted run first or in the middle: each block read as transposed
    # matrices (one per entry of the legs before the run), with the sign of
    # moving the run behind the legs after it
    ("z2", [(64, 64, 1), (40, 24, 0), (33, 31, 0)], [(64, 64, 0), (20, 12, 1)], [0], [0], True),
    ("z2", [(6, 5, 0), (64, 64, 1), (40, 24, 0), (16, 12, 0)], [(64, 64, 0), (20, 12, 1)], [1], [0], True),
    ("z2g", [(6, 5, 0), (64, 64, 1), (40, 24, 0), (16, 12, 0)], [(64, 64, 0), (20, 12, 1)], [1], [0], True),
    ("u1", [((3, 4, 2), 0), ((64, 48), 1), ((3,), 1), ((16, 16), 0), ((24, 32, 16), 0)],
     [((64, 48), 0), ((3,), 0), ((5, 6, 7), 1)], [1, 2], [0, 1], True),
    # two contracted combinations per group, contracted legs not one run, or
    # row groups far shorter than a tile: A is copied
    ("z2", [(40, 24, 0), (64, 64, 1), (6, 5, 1)], [(64, 64, 0), (6, 5, 0), (20, 12, 1)], [1, 2], [0, 1], False),
    ("z2", [(40, 24, 0), (64, 64, 1), (33, 31, 0), (6, 5, 1)], [(6, 5, 0), (64, 64, 0), (20, 12, 1)], [1, 3], [1, 0],
     False),
    ("z2", [(3, 2, 0), (2, 3, 0), (64, 64, 1)], [(64, 64, 0), (20, 12, 1)], [2], [0], False),
    ("z2", [(64, 64, 0), (32, 32, 1), (4, 4, 0)], [(32, 32, 0), (20, 12, 1)], [1], [0], False),
])
def test_ftensordot_reads_a_in_place(P, case):
    name, la, lb, ax_a, ax_b, in_place = case
    rng = np.random.default_rng(len(name) + 7 * len(la) + 3 * sum(ax_a) + len(lb))
    if name.startswith("z2"):
        sym = S.Z2
        mk = lambda e, o, du: make_leg(sym, [(0,), (1,)], [e, o], du)
        legs_a, legs_b = [mk(*l) for l in la], [mk(*l) for l in lb]
    else:
        sym = S.U1
        legs_a = [_u1_leg(d, du, (0, 1) if len(d) == 2 else (-1, 0, 1) if len(d) == 3 else (0,)) for d, du in la]
        legs_b = [_u1_leg(d, du, (0, 1) if len(d) == 2 else (-1, 0, 1) if len(d) == 3 else (0,)) for d, du in lb]
    A = rand_tensor(rng, sym, legs_a, total=S.zero(sym))
    B = rand_tensor(rng, sym, legs_b, total=S.zero(sym))
    conv = "global" if name.endswith("g") else "local"
    from paper_2410_02215_amd import ftn
    ref = ftensordot(A, B, ax_a, ax_b, conv=conv)
    ga, gb = to_gpu(A), to_gpu(B)
    pc = P.LOCAL if conv == "local" else P.GLOBAL
    P.ftensordot(ga, gb, ax_a, ax_b, conv=pc)  # builds and caches the plan
    torch.cuda.synchronize()
    ftn.profile_collect()
    ftn.profile_enable(True)
    G = P.ftensordot(ga, gb, ax_a, ax_b, conv=pc)
    torch.cuda.synchronize()
    ftn.profile_enable(False)
    # one signed permute (B's) when A is read in place, else two
    assert ftn.profile_collect()["permute"][1] == (1 if in_place else 2)
    assert_same_structure(ref, G)
    r = flat_blocks(ref)
    np.testing.assert_allclose(_data(G), r, rtol=0, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("gemm", ["f32", "bf16x3"])
@pytest.mark.parametrize("conv", ["local", "global"])
def test_ftensordot_reads_a_in_place_fp32_forms(P, gemm, conv):
    # the FP32 and split-BF16 kernels on A read in place as signed transposed
    # blocks (and as row slabs), against the oracle on the FP32-rounded inputs
    rng = np.random.default_rng(61 + len(gemm) + len(conv))
    sym = S.Z2
    mk = lambda e, o, du: make_leg(sym, [(0,), (1,)], [e, o], du)
    tol = {"f32": 1e-6, "bf16x3": 1e-4}[gemm]
    from paper_2410_02215_amd import ftn
    for la, lb, ax in [([(6, 5, 0), (64, 64, 1), (40, 24, 0), (16, 12, 0)], [(64, 64, 0), (20, 12, 1)], [1]),
                       ([(40, 24, 0), (33, 31, 0), (64, 64, 1)], [(64, 64, 0), (20, 12, 1)], [2])]:
        A = rand_tensor(rng, sym, [mk(*l) for l in la], total=(0,))
        B = rand_tensor(rng, sym, [mk(*l) for l in lb], total=(1,))
        A32, B32 = rounded_f32(A), rounded_f32(B)
        ref = ftensordot(A32, B32, ax, [0], conv=conv)
        ga, gb = to_gpu(A, torch.float32), to_gpu(B, torch.float32)
        pc = P.LOCAL if conv == "local" else P.GLOBAL
        gk = P.GEMM_F32 if gemm == "f32" else P.GEMM_BF16X3
        P.ftensordot(ga, gb, ax, [0], conv=pc, gemm=gk)
        torch.cuda.synchronize()
        ftn.profile_collect()
        ftn.profile_enable(True)
        G = P.ftensordot(ga, gb, ax, [0], conv=pc, gemm=gk)
        torch.cuda.synchronize()
        ftn.profile_enable(False)
        assert ftn.profile_collect()["permute"][1] == 1
        assert_same_structure(ref, G)
        r = flat_blocks(ref)
        err = np.abs(_data(G) - r).max() / np.abs(r).max()
        assert err < tol, err


@pytest.mark.parametrize("gemm", ["f32", "bf16x3"])
def test_ftensordot_fp32_forms(P, gemm):
    # FP32 tensors hold the FP64 inputs rounded to nearest; the oracle runs on
    # the same rounded values (promoted to FP64), so the error measured is that
    # of the FP32 or split-BF16 arithmetic, relative to the largest entry
    rng = np.random.default_rng(8)
    sym = S.U1U1
    tol = {"f32": 1e-6, "bf16x3": 1e-4}[gemm]
    worst = 0.0
    for trial in range(6):
        k = int(rng.integers(1, 3))
        A, B, ax_a, ax_b = _rand_pair(rng, sym, k, 2, 2, 4)
        A32, B32 = rounded_f32(A), rounded_f32(B)
        ref = ftensordot(A32, B32, ax_a, ax_b, conv="local")
        Ga = to_gpu(A, torch.float32)
        Gb = to_gpu(B, torch.float32)
        G = P.ftensordot(Ga, Gb, ax_a, ax_b, gemm=P.GEMM_F32 if gemm == "f32" else P.GEMM_BF16X3)
        assert_same_structure(ref, G)
        r = flat_blocks(ref)
        err = np.abs(_data(G) - r).max(initial=0) / max(np.abs(r).max(initial=0), 1e-30)
        worst = max(worst, err)
        assert err < tol, err
    print("%s ftensordot: max error %.3g of the largest entry" % (gemm, worst))


def test_errors_are_reported(P):
    rng = np.random.default_rng(9)
    sym = S.Z2
    la = rand_leg(rng, sym)
    A = rand_tensor(rng, sym, [la, rand_leg(rng, sym)])
    B = rand_tensor(rng, sym, [la, rand_leg(rng, sym)])  # same dual: not contractible
    with pytest.raises(P.FtnError) as e:
        P.ftensordot(to_gpu(A), to_gpu(B), [0], [0])
    assert e.value.code == -2
    with pytest.raises(P.FtnError) as e:
        P.ftranspose(to_gpu(A), [0, 0])
    assert e.value.code == -1


def test_memory_statistics_follow_allocations(P):
    # one Z2 tensor of 2 x (1024 x 1024) FP64 entries: 16 MiB of block data
    dev = torch.cuda.current_device()
    torch.cuda.synchronize()
    s0 = P.ftn.memory_stats(dev, reset_peak=True)  # values before the reset
    assert s0["peak"] >= s0["in_use"] and s0["reserved"] >= s0["in_use"] >= 0
    assert P.ftn.memory_stats(dev)["peak"] == s0["in_use"]
    legs = [([(0, 0), (1, 0)], [1024, 1024], 0), ([(0, 0), (1, 0)], [1024, 1024], 1)]
    G = P.Tensor.create(0, legs, (0, 0))
    s1 = P.ftn.memory_stats(dev)
    assert s1["in_use"] - s0["in_use"] >= 2 * 1024 * 1024 * 8
    assert s1["peak"] >= s1["in_use"] and s1["reserved"] >= s1["in_use"]
    del G
    torch.cuda.synchronize()
    s2 = P.ftn.memory_stats(dev)
    assert s2["in_use"] <= s1["in_use"] - 2 * 1024 * 1024 * 8
    assert s2["peak"] == s1["peak"]
    s3 = P.ftn.memory_stats(dev, reset_peak=True)
    assert s3["peak"] == s1["peak"]
    assert P.ftn.memory_stats(dev)["peak"] == s3["in_use"]
    with pytest.raises(P.FtnError) as e:
        P.ftn.memory_stats(-1)
    assert e.value.code == -1


def test_compress_bond_with_no_common_sector(P):
    # the two ends share no charge that carries blocks on both sides: F(AB)
    # is zero across the bond, nothing is kept and the bond leg is emptied on
    # both tensors (the oracle's compress_bond gives the same structure)
    from oracle.linalg import compress_bond
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    rng = np.random.default_rng(11)
    A = rand_tensor(rng, sym, [l(3, 2, 0), l(4, 5, 1)], total=(0,))
    A.blocks = {k: v for k, v in A.blocks.items() if k[1] == 0}   # even bond sector only
    B = rand_tensor(rng, sym, [l(4, 5, 0)], total=(1,))           # odd bond sector only
    A2, B2, info = compress_bond(A, B, 1, 0, 3)
    assert A2.legs[1].charges == () and B2.legs[0].charges == ()
    Ga = P.Tensor.from_dense(0, [([(0, 0), (1, 0)], [3, 2], 0), ([(0, 0)], [4], 1)], (0, 0),
                             torch.from_numpy(A.to_dense()[:, :4].copy()).cuda())
    Gb = P.Tensor.from_dense(0, [([(1, 0)], [5], 0)], (1, 0), torch.from_numpy(B.to_dense()[4:].copy()).cuda())
    ga, gb, info = P.compress_bond(Ga, Gb, 1, 0, 3)
    assert ga.leg(1)[0] == [] and gb.leg(0)[0] == []
    assert ga.size == 0 and gb.size == 0 and len(info["svals"]) == 0


def test_torch_owns_the_library_memory(P):
    # with torch's caching allocator registered, tensor data and temporaries
    # of a contraction come from torch (its allocated bytes grow while the
    # library's own cache does not), results are unchanged, and blocks made
    # by either allocator go back to it after the other is registered
    from tests.helpers import rand_tensor as rt
    rng = np.random.default_rng(12)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rt(rng, sym, [l(64, 48, 0), l(40, 30, 1)], total=(0,))
    B = rt(rng, sym, [l(40, 30, 0), l(50, 20, 1)], total=(0,))
    ref = flat_blocks(ftensordot(A, B, [1], [0], conv="local"))
    dev = torch.cuda.current_device()
    G0 = to_gpu(A)                                   # built-in allocator
    torch.cuda.synchronize()
    lib0 = P.ftn.memory_stats(dev)["in_use"]
    t0 = torch.cuda.memory_allocated()
    try:
        P.ftn.use_torch_allocator(True)
        Ga, Gb = to_gpu(A), to_gpu(B)
        C = P.ftensordot(Ga, Gb, [1], [0])
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - t0 >= 8 * (Ga.size + Gb.size + C.size)
        assert P.ftn.memory_stats(dev)["in_use"] == lib0
        np.testing.assert_allclose(C.data().cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        C2 = P.ftensordot(G0, Gb, [1], [0])          # a built-in block used beside torch's
        np.testing.assert_allclose(C2.data().cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        del G0                                       # back to the built-in cache
    finally:
        P.ftn.use_torch_allocator(False)
    torch.cuda.synchronize()
    del Ga, Gb, C, C2                                # back to torch
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= t0


def test_profiler_kernel_classes_add_up_to_their_families(P):
    # the per-kernel classes of the grouped GEMM and of the factorisation
    # kernels partition their families' time, launches and work
    from paper_2410_02215_amd import ftn
    rng = np.random.default_rng(33)
    sym = S.Z2
    l = lambda e, o, d: make_leg(sym, [(0,), (1,)], [e, o], d)
    A = rand_tensor(rng, sym, [l(90, 70, 0), l(150, 130, 1)], total=(0,))
    B = rand_tensor(rng, sym, [l(150, 130, 0), l(200, 180, 1)], total=(0,))
    ga, gb = to_gpu(A), to_gpu(B)
    torch.cuda.synchronize()
    ftn.profile_collect()
    ftn.profile_enable(True)
    P.ftensordot(ga, gb, [1], [0])
    P.compress_bond(ga, gb, 1, 0, 40)
    torch.cuda.synchronize()
    ftn.profile_enable(False)
    pr = ftn.profile_collect()
    gk = [k for k in ftn.PROF_CLASSES if k.startswith("k_gemm_f64_")] + ["k_skinny_f64"]
    fk = ["k_orth_factor", "k_jacobi_sweep", "k_jacobi_sweep_la", "k_jacobi_vectors", "k_svd_cols"]
    assert pr["gemm_f64"][1] > 0 and pr["factor"][1] > 0
    ms = sum(pr[k][0] for k in gk) + pr["k_splitk_reduce_f64"][0]
    assert abs(ms - pr["gemm_f64"][0]) <= 1e-6 * pr["gemm_f64"][0] + 1e-9
    assert sum(pr[k][1] for k in gk) == pr["gemm_f64"][1]
    assert abs(sum(pr[k][2] for k in gk) - pr["gemm_f64"][2]) <= 1e-9 * pr["gemm_f64"][2]
    assert abs(sum(pr[k][0] for k in fk) - pr["factor"][0]) <= 1e-6 * pr["factor"][0] + 1e-9
    assert sum(pr[k][1] for k in fk if k != "k_jacobi_vectors") == pr["factor"][1]
