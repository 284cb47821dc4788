"""The grouped-GEMM tile autotuner (``ftn_autotune``) on the device.

Tuning mode times the candidate tile shapes of an unseen plan and stores the
fastest; contractions planned with tuned shapes still agree with the oracle
at the FP64 tolerance; a saved table loads back and serves later plans of the
same shape key without tuning.
"""

import json
import os

import numpy as np
import pytest
import torch

from oracle import symmetry as S
from oracle.ops import ftensordot
from oracle.tensor import make_leg
from tests.helpers import rand_tensor
from tests.gpu_helpers import to_gpu, flat_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2410_02215_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    P.load_library()
    yield P
    P.ftn.autotune(0)


def _pair(rng, dims_a, dims_k, dims_b):
    l = lambda d, dual: make_leg(S.Z2, [(0,), (1,)], d, dual)
    A = rand_tensor(rng, S.Z2, [l(dims_a, 0), l(dims_k, 1)], total=(0,))
    B = rand_tensor(rng, S.Z2, [l(dims_k, 0), l(dims_b, 1)], total=(0,))
    return A, B


def test_tuned_contractions_match_oracle_and_table_round_trips(P, tmp_path):
    rng = np.random.default_rng(900)
    try:
        P.ftn.autotune(2)
        st0 = P.ftn.autotune_stats()
        for dims in (((700, 513), (300, 129), (640, 97)), ((40, 3000), (17, 250), (2900, 33))):
            A, B = _pair(rng, *dims)
            ref = flat_blocks(ftensordot(A, B, [1], [0], conv="local"))
            G = P.ftensordot(to_gpu(A), to_gpu(B), [1], [0])
            got = G.data().cpu().numpy()
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        st1 = P.ftn.autotune_stats()
        assert st1["tuned"] >= st0["tuned"] + 2
        path = os.path.join(str(tmp_path), "tune.json")
        P.ftn.autotune_save(path)
        entries = json.load(open(path))["entries"]
        assert len(entries) == st1["entries"] and all(len(v) == 3 for v in entries.values())
        # a fresh table entry set loads back; mode 1 serves plans of the same
        # shape key from it without tuning
        P.ftn.autotune_load(path)
        P.ftn.autotune(1)
        A, B = _pair(rng, (701, 512), (301, 128), (641, 96))
        ref = flat_blocks(ftensordot(A, B, [1], [0], conv="local"))
        G = P.ftensordot(to_gpu(A), to_gpu(B), [1], [0])
        np.testing.assert_allclose(G.data().cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        st2 = P.ftn.autotune_stats()
        assert st2["tuned"] == st1["tuned"] and st2["hits"] > st1["hits"]
    finally:
        P.ftn.autotune(0)
