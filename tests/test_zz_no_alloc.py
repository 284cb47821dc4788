"""The allocation-free contraction ``ftn_ftensordot_noalloc`` against
``ftn_ftensordot``: the same plan and kernels with the temporaries in the
library's fixed per-GPU scratch array, so the outputs agree bit for bit; two
calls in a row, the second on a smaller contraction; the library's caching
allocator does not move during the calls; errors for an uncached plan, a
wrong output size and temporaries beyond the scratch array; products whose
A is read in place (row slabs, transposed blocks) needing only B's copy in
the array.
"""

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from tests.helpers import rand_tensor
from tests.gpu_helpers import to_gpu
from oracle.tensor import make_leg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2410_02215_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    P.load_library()
    return P


def _pair(rng, sym, dims_free_a, dims_k, dims_free_b):
    qs = [(0,), (1,)] if sym == S.Z2 else [(-1,), (0,), (1,)]
    mk = lambda d, dual: make_leg(sym, qs, d, dual)
    A = rand_tensor(rng, sym, [mk(dims_free_a, 0), mk(dims_k, 1)], total=S.zero(sym))
    B = rand_tensor(rng, sym, [mk(dims_k, 0), mk(dims_free_b, 1)], total=S.zero(sym))
    return A, B


@pytest.mark.parametrize("dtype,gemm", [("f64", 0), ("f32", 1), ("f32", 2)])
def test_noalloc_matches_ftensordot_on_two_calls(P, dtype, gemm):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(700)
    dev = torch.cuda.current_device()
    cases = [_pair(rng, S.Z2, [300, 257], [190, 77], [211, 160]),   # several tiles, ragged tails
             _pair(rng, S.U1, [20, 13, 9], [7, 11, 5], [16, 3, 12])]  # the smaller second call
    for A, B in cases:
        Ga, Gb = to_gpu(A, tdt), to_gpu(B, tdt)
        ref = P.ftensordot(Ga, Gb, [1], [0], gemm=gemm)           # caches the plan
        want = ref.data().clone()
        out = torch.full((ref.size,), float("nan"), device="cuda", dtype=tdt)
        torch.cuda.synchronize()
        before = P.ftn.memory_stats(dev)
        P.ftensordot_noalloc(Ga, Gb, [1], [0], out, gemm=gemm)
        torch.cuda.synchronize()
        after = P.ftn.memory_stats(dev)
        assert after["reserved"] == before["reserved"] and after["in_use"] == before["in_use"]
        assert torch.equal(out, want), (out - want).abs().max().item()


def test_noalloc_errors(P):
    rng = np.random.default_rng(701)
    A, B = _pair(rng, S.Z2, [5, 4], [3, 6], [2, 7])
    Ga, Gb = to_gpu(A), to_gpu(B)
    out = torch.zeros(1000, device="cuda", dtype=torch.float64)
    with pytest.raises(P.FtnError) as e:                          # no cached plan yet
        P.ftensordot_noalloc(Ga, Gb, [1], [0], out, gemm=0, conv=P.GLOBAL)
    assert e.value.code == -6
    ref = P.ftensordot(Ga, Gb, [1], [0], conv=P.GLOBAL)
    with pytest.raises(P.FtnError) as e:                          # wrong output size
        P.ftensordot_noalloc(Ga, Gb, [1], [0], out[:ref.size - 1], conv=P.GLOBAL)
    assert e.value.code == -1
    # A's fused copy, 2 x 4096 x 1200 FP64 (two contracted sector combinations
    # per charge, so its blocks cannot be read in place), exceeds the 64 MiB array
    two = [(0, 0), (1, 0)]
    big_a = P.Tensor.create(0, [(two, [4096, 4096], 0), (two, [600, 600], 1), (two, [1, 1], 1)], (0, 0))
    big_b3 = P.Tensor.create(0, [(two, [600, 600], 0), (two, [1, 1], 0), (two, [8, 8], 1)], (0, 0))
    c = P.ftensordot(big_a, big_b3, [1, 2], [0, 1])
    o2 = torch.zeros(c.size, device="cuda", dtype=torch.float64)
    with pytest.raises(P.FtnError) as e:
        P.ftensordot_noalloc(big_a, big_b3, [1, 2], [0, 1], o2)
    assert e.value.code == -1
    big_b = P.Tensor.create(0, [(two, [1200, 1200], 0), (two, [8, 8], 1)], (0, 0))
    # with A's contracted leg last A's blocks are read in place: only B's fused
    # copy takes scratch space, so the same product at that size fits
    big_a2 = P.Tensor.create(0, [([(0, 0), (1, 0)], [4096, 4096], 0), ([(0, 0), (1, 0)], [1200, 1200], 1)], (0, 0))
    g = torch.Generator(device="cuda").manual_seed(702)
    big_a2.data_view().normal_(generator=g)
    big_b.data_view().normal_(generator=g)
    torch.cuda.synchronize()
    c2 = P.ftensordot(big_a2, big_b, [1], [0])
    want = c2.data()
    o3 = torch.full((c2.size,), float("nan"), device="cuda", dtype=torch.float64)
    P.ftensordot_noalloc(big_a2, big_b, [1], [0], o3)
    torch.cuda.synchronize()
    assert torch.equal(o3, want) and want.abs().max().item() > 0
    # the contracted leg first: A's blocks read in place as transposed matrices
    big_a3 = P.Tensor.create(0, [(two, [1200, 1200], 1), (two, [4096, 4096], 0)], (0, 0))
    big_a3.data_view().normal_(generator=g)
    torch.cuda.synchronize()
    c3 = P.ftensordot(big_a3, big_b, [0], [0])
    want = c3.data()
    o4 = torch.full((c3.size,), float("nan"), device="cuda", dtype=torch.float64)
    P.ftensordot_noalloc(big_a3, big_b, [0], [0], o4)
    torch.cuda.synchronize()
    assert torch.equal(o4, want) and want.abs().max().item() > 0
