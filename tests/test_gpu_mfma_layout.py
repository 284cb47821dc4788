"""Lane layout of the 16x16x4 MFMA builtins used by the grouped GEMM.

Probe: A = e_0-column with values i+1, B = e_0-row with values 100(j+1), so
D[i][j] = 100 (i+1)(j+1) identifies the (row, col) each lane/item holds.
The GEMM kernel relies on: inputs A[lane%16][lane/16], B[lane/16][lane%16];
output item r of lane l is D[row][l%16] with row = 4*(l/16) + r for FP32 and
row = l/16 + 4*r for FP64.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("probe") / "mfma_probe.so")
    src = os.path.join(HERE, "probes", "mfma_layout.hip")
    subprocess.run(["hipcc", "-O2", "--offload-arch=gfx950", "-shared", "-fPIC", src, "-o", out], check=True)
    return ctypes.CDLL(out)


def _maps(vals):
    """(row, col) held by item r of lane l, decoded from 1000 (i+1) + (j+1)."""
    rows = np.zeros((64, 4), dtype=int)
    cols = np.zeros((64, 4), dtype=int)
    for l in range(64):
        for r in range(4):
            v = int(round(vals[l * 4 + r]))
            rows[l, r] = v // 1000 - 1
            cols[l, r] = v % 1000 - 1
    return rows, cols


def test_mfma_output_layout(probe):
    h64 = (ctypes.c_double * 256)()
    h32 = (ctypes.c_float * 256)()
    assert probe.run_probe(h64, h32) == 0
    lanes = np.arange(64)[:, None]
    items = np.arange(4)[None, :]
    exp_cols = np.broadcast_to(lanes % 16, (64, 4))
    for name, h in (("f32", h32), ("f64", h64)):
        exp_rows = 4 * (lanes // 16) + items if name == "f32" else lanes // 16 + 4 * items
        rows, cols = _maps(np.array(h[:]))
        print(name, "rows of lanes 0,16,32,48:", rows[[0, 16, 32, 48]].tolist(),
              "cols of lanes 0,1,16:", cols[[0, 1, 16]].tolist())
        np.testing.assert_array_equal(rows, exp_rows, err_msg=name + " rows")
        np.testing.assert_array_equal(cols, exp_cols, err_msg=name + " cols")
