"""Write synth/data/paths.json: seeded contraction paths of the workloads.

The paths are inputs shared by the oracle and the library. Each is the best
(lowest peak intermediate size, then lowest flop count) of one deterministic
and many Boltzmann-sampled greedy paths (synth.paths.best_of_greedy), with
every bra tensor first paired with its ket partner.

    python -m synth.make_paths
"""

import json
import os

from . import workloads as W
from .paths import best_of_greedy, path_stats

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "data", "paths.json")


def _first_pairs(spec, op_sites):
    n = spec.n_sites
    first = []
    if op_sites is not None:
        u, v = op_sites
        first += [(n + u, 2 * n), (n + v, n + u), (u, n + u), (v, n + u)]
    first += [(s, n + s) for s in range(n) if op_sites is None or s not in op_sites]
    return first


def plan(spec, chi, op_sites=None, seed=7, trials=3000, temperature=2.0):
    n = spec.n_sites
    nt = 2 * n + (1 if op_sites is not None else 0)
    bonds = [(t1, t2, d) for (t1, _, t2, _, d) in W.norm_network_bonds(spec, op_sites)]
    p = best_of_greedy(nt, bonds, chi=chi, seed=seed, first_pairs=_first_pairs(spec, op_sites),
                       trials=trials, temperature=temperature)
    st = path_stats(nt, bonds, p, chi=chi)
    return dict(path=[list(x) for x in p],
                log2_flops=[s["lflops"] for s in st],
                peak_log2_size=max(max(s["lz"], s["lx"], s["ly"]) for s in st))


def main():
    out = {}
    cfg = W.c2()
    out["c2_norm"] = plan(cfg["spec"], cfg["chi"], seed=7, temperature=2.0)
    out["c2_hop"] = plan(cfg["spec"], cfg["chi"], op_sites=cfg["op_sites"], seed=14, temperature=1.5)
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    for k, v in out.items():
        print(k, "steps", len(v["path"]), "peak log2 size", v["peak_log2_size"],
              "log2 flops", round(max(v["log2_flops"]), 2))


if __name__ == "__main__":
    main()
