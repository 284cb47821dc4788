"""Write tests/golden/values.json with oracle values of the full workloads.

Calls only the oracle (and the seeded inputs of synth). Each entry records
the network value as (mantissa, exp2) with value = mantissa * 2**exp2.

    python -m tests.golden.make_golden
"""

import hashlib
import json
import os
import time

import torch

from oracle import physics as OP
from oracle.network import network_value
from synth import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "values.json")


def _hash(path):
    return hashlib.sha1(json.dumps(path).encode()).hexdigest()[:12]


def main():
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    paths = json.load(open(os.path.join(ROOT, "synth", "data", "paths.json")))
    out = {}
    cfg = W.c1()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    p = W.norm_path(spec, seed=0)
    m, e = network_value(OP.norm_network(spec, kets, conv="global"), p)
    out["c1_norm"] = dict(mantissa=m, exp2=e, path=p, note="exact, global convention")
    cfg = W.c2()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    t0 = time.time()
    pn = paths["c2_norm"]["path"]
    m, e = network_value(OP.norm_network(spec, kets, conv="local"), pn, chi=cfg["chi"])
    out["c2_norm"] = dict(mantissa=m, exp2=e, path_sha=_hash(pn), chi=cfg["chi"], seconds=time.time() - t0)
    from synth.operators import operator_dense
    from oracle.tensor import FTensor
    G = OP.operator_tensor(OP.two_site_local("hop"), kets[0].legs[0], "Z2")
    ph = paths["c2_hop"]["path"]
    t0 = time.time()
    m, e = network_value(OP.norm_network(spec, kets, op=G, op_sites=cfg["op_sites"], conv="local"), ph,
                         chi=cfg["chi"])
    out["c2_hop"] = dict(mantissa=m, exp2=e, path_sha=_hash(ph), chi=cfg["chi"], op_sites=list(cfg["op_sites"]),
                         seconds=time.time() - t0)
    # the precision workload's structure on a 16-site (2 x 2 x 2 cells) diamond
    # cluster at chi = 32: the largest cluster the oracle contracts in minutes
    # (the 64-site chi = 128 workload is beyond it); bonds reach 700 per sector
    # before compression
    cfg = W.c3(cells=(2, 2, 2), chi=32)
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    p3 = W.norm_path(spec, chi=32, seed=0)
    t0 = time.time()
    m, e = network_value(OP.norm_network(spec, kets, conv="local"), p3, chi=32)
    out["c3_222_norm"] = dict(mantissa=m, exp2=e, path_sha=_hash(p3), chi=32, cells=[2, 2, 2],
                              seconds=time.time() - t0)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "path"} for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main()
