"""Write tests/golden/values.json with oracle values of the full workloads.

Calls only the oracle (and the seeded inputs of synth). Each entry records
the network value as (mantissa, exp2) with value = mantissa * 2**exp2.

    python -m tests.golden.make_golden            # every entry
    python -m tests.golden.make_golden c5_hop_grad  # the named entries only

The gradient entry stores, per tensor of the network (ids: bra s -> s, ket
s -> n + s, operator -> 2 n), the squared norm of d(value)/dT and its inner
product with a probe R_T whose entries (blocks flattened in key order) are
numpy.random.default_rng(PROBE_SEED + id).standard_normal.
"""

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

import torch

from oracle import physics as OP
from oracle.network import network_value
from synth import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "values.json")
PROBE_SEED = 7000


def _hash(path):
    return hashlib.sha1(json.dumps(path).encode()).hexdigest()[:12]


def c1_norm():
    cfg = W.c1()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    p = W.norm_path(spec, seed=0)
    m, e = network_value(OP.norm_network(spec, kets, conv="global"), p)
    return dict(mantissa=m, exp2=e, path=p, note="exact, global convention")


def _c2():
    paths = json.load(open(os.path.join(ROOT, "synth", "data", "paths.json")))
    cfg = W.c2()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    return paths, cfg, spec, kets


def c2_norm():
    paths, cfg, spec, kets = _c2()
    t0 = time.time()
    pn = paths["c2_norm"]["path"]
    m, e = network_value(OP.norm_network(spec, kets, conv="local"), pn, chi=cfg["chi"])
    return dict(mantissa=m, exp2=e, path_sha=_hash(pn), chi=cfg["chi"], seconds=time.time() - t0)


def c2_hop():
    paths, cfg, spec, kets = _c2()
    G = OP.operator_tensor(OP.two_site_local("hop"), kets[0].legs[0], "Z2")
    ph = paths["c2_hop"]["path"]
    t0 = time.time()
    m, e = network_value(OP.norm_network(spec, kets, op=G, op_sites=cfg["op_sites"], conv="local"), ph,
                         chi=cfg["chi"])
    return dict(mantissa=m, exp2=e, path_sha=_hash(ph), chi=cfg["chi"], op_sites=list(cfg["op_sites"]),
                seconds=time.time() - t0)


def c3_222_norm():
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
    return dict(mantissa=m, exp2=e, path_sha=_hash(p3), chi=32, cells=[2, 2, 2], seconds=time.time() - t0)


def c5_hop_grad():
    # value and gradient of <psi|h_(13,14)|psi> (hopping term) on the 6 x 6
    # differentiation lattice at chi = 32, absorbed layer by layer: two of its
    # compressions have bond sectors of 256
    from oracle.adjoint import network_grad
    from oracle.tensor import FTensor, Leg
    from oracle import symmetry as S
    from synth.operators import operator_dense
    cfg = W.c5()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    phys = kets[0].legs[0]
    out_l, in_l = phys, Leg(phys.charges, phys.dims, 1)
    sites = (13, 14)
    G = FTensor.from_dense(S.Z2, [out_l, out_l, in_l, in_l], (0,), operator_dense("hop", "Z2"))
    net = OP.norm_network(spec, kets, op=G, op_sites=sites, conv="local")
    path = W.norm_layer_path(spec, cfg["lx"], cfg["ly"], sites)
    t0 = time.time()
    v, grads = network_grad(net, path, chi=cfg["chi"])
    m, e = math.frexp(v)
    g2, proj = [], []
    for t in sorted(grads):
        T = grads[t]
        parts = [T.block(k).detach().numpy().ravel() for k in T.keys()]
        g = np.concatenate(parts) if parts else np.zeros(0)
        r = np.random.default_rng(PROBE_SEED + t).standard_normal(g.size)
        g2.append(float(g @ g))
        proj.append(float(g @ r))
    return dict(mantissa=m, exp2=e, chi=cfg["chi"], op_sites=list(sites), path_sha=_hash(path), grad_sq=g2,
                grad_probe=proj, seconds=time.time() - t0)


ENTRIES = {"c1_norm": c1_norm, "c2_norm": c2_norm, "c2_hop": c2_hop, "c3_222_norm": c3_222_norm,
           "c5_hop_grad": c5_hop_grad}


def main(names=None):
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    out = json.load(open(OUT)) if names and os.path.exists(OUT) else {}
    for k in names or list(ENTRIES):
        out[k] = ENTRIES[k]()
        print(k, "done", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk not in ("path", "grad_sq", "grad_probe")}
                      for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:] or None)
