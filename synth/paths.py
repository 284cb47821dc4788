"""Seeded greedy contraction-path planner (an input to both sides).

The paper chooses contraction trees with hyperoptimized searches over the
tensor network graph alone, since fermionic signs add no cost to the search
(Sec. III). That search is prior art; this module stands in for it with a
deterministic greedy planner: repeatedly contract the connected pair that
minimises ``log2 size(out) - log2 size(X) - log2 size(Y)``, where the bonds an
intermediate shares with one neighbour are merged into one bond whose
dimension is the product, capped at ``chi`` when the product exceeds it
(compression as early as possible, Sec. III). Ties are broken by
``numpy.random.default_rng(seed)``.

The path is returned in SSA form: inputs are ids ``0..n-1`` and the k-th
contraction creates id ``n + k``.
"""

import math

import numpy as np


def _logsize(bonds_of, dims, t):
    s = 0.0
    for b in bonds_of[t]:
        s += math.log2(dims[b])
    return s


def greedy_path(n_tensors, bonds, open_dims=None, chi=None, seed=0,
                first_pairs=(), temperature=0.0):
    """Plan a contraction path.

    ``bonds``: list of ``(t1, t2, dim)``; ``open_dims``: per-tensor list of
    open-leg dims (contribute to sizes only). ``first_pairs``: pairs of input
    ids contracted first, in the given order, before the greedy search.
    Returns a list of SSA pairs ``(i, j)``.
    """
    rng = np.random.default_rng(seed)
    dims = {}
    ends = {}
    bonds_of = {t: set() for t in range(n_tensors)}
    for b, (t1, t2, d) in enumerate(bonds):
        dims[b] = float(d)
        ends[b] = [t1, t2]
        bonds_of[t1].add(b)
        bonds_of[t2].add(b)
    opens = {t: 0.0 for t in range(n_tensors)}
    if open_dims is not None:
        for t, od in enumerate(open_dims):
            opens[t] = sum(math.log2(d) for d in od)
    next_id = n_tensors
    path = []
    alive = set(range(n_tensors))

    def neighbours(t):
        out = {}
        for b in bonds_of[t]:
            o = ends[b][0] if ends[b][1] == t else ends[b][1]
            out.setdefault(o, []).append(b)
        return out

    def contract(x, y):
        nonlocal next_id
        z = next_id
        next_id += 1
        shared = bonds_of[x] & bonds_of[y]
        new_bonds = (bonds_of[x] | bonds_of[y]) - shared
        for b in shared:
            del dims[b]
            del ends[b]
        bonds_of[z] = set()
        # merge parallel bonds to each neighbour
        per_nb = {}
        for b in new_bonds:
            o = ends[b][0] if ends[b][1] in (x, y) else ends[b][1]
            per_nb.setdefault(o, []).append(b)
        for o, bl in per_nb.items():
            d = 1.0
            for b in bl:
                d *= dims[b]
                bonds_of[o].discard(b)
                del dims[b]
                del ends[b]
            if chi is not None and d > chi:
                d = float(chi)
            nb = ("m", z, o, len(path))
            dims[nb] = d
            ends[nb] = [z, o]
            bonds_of[z].add(nb)
            bonds_of[o].add(nb)
        opens[z] = opens[x] + opens[y]
        del bonds_of[x]
        del bonds_of[y]
        alive.discard(x)
        alive.discard(y)
        alive.add(z)
        path.append((x, y))
        return z

    def logsize(t):
        return _logsize(bonds_of, dims, t) + opens[t]

    ssa_of = {t: t for t in range(n_tensors)}
    for a, b in first_pairs:
        z = contract(ssa_of[a], ssa_of[b])
        ssa_of[a] = z
        ssa_of[b] = z

    while len(alive) > 1:
        best = None
        for x in sorted(alive):
            nbs = neighbours(x)
            for y in sorted(nbs):
                if y <= x:
                    continue
                # size of the merged result
                ls = opens[x] + opens[y]
                nx = neighbours(x)
                ny = neighbours(y)
                merged = {}
                for o, bl in list(nx.items()) + list(ny.items()):
                    if o in (x, y):
                        continue
                    merged.setdefault(o, 0.0)
                    merged[o] += sum(math.log2(dims[b]) for b in bl)
                for o, l in merged.items():
                    if chi is not None and l > math.log2(chi):
                        l = math.log2(chi)
                    ls += l
                score = ls - logsize(x) - logsize(y)
                if temperature > 0.0:
                    # Gumbel perturbation = Boltzmann sampling over scores
                    g = -math.log(-math.log(max(rng.random(), 1e-300)))
                    key = (score - temperature * g, 0.0)
                else:
                    key = (round(score, 9), rng.random())
                if best is None or key < best[0]:
                    best = (key, x, y)
        if best is None:
            # disconnected remainder: outer products in id order
            xs = sorted(alive)
            contract(xs[0], xs[1])
            continue
        contract(best[1], best[2])
    return path


def path_stats(n_tensors, bonds, path, open_dims=None, chi=None):
    """Predicted log2 sizes of each intermediate (planning estimate only)."""
    dims = {}
    ends = {}
    bonds_of = {t: set() for t in range(n_tensors)}
    for b, (t1, t2, d) in enumerate(bonds):
        dims[b] = float(d)
        ends[b] = [t1, t2]
        bonds_of[t1].add(b)
        bonds_of[t2].add(b)
    opens = {t: 0.0 for t in range(n_tensors)}
    if open_dims is not None:
        for t, od in enumerate(open_dims):
            opens[t] = sum(math.log2(d) for d in od)
    nid = n_tensors
    out = []
    for (x, y) in path:
        z = nid
        nid += 1
        shared = bonds_of[x] & bonds_of[y]
        lk = sum(math.log2(dims[b]) for b in shared)
        lx = sum(math.log2(dims[b]) for b in bonds_of[x]) + opens[x]
        ly = sum(math.log2(dims[b]) for b in bonds_of[y]) + opens[y]
        new_bonds = (bonds_of[x] | bonds_of[y]) - shared
        for b in shared:
            del dims[b]
            del ends[b]
        per_nb = {}
        for b in new_bonds:
            o = ends[b][0] if ends[b][1] in (x, y) else ends[b][1]
            per_nb.setdefault(o, []).append(b)
        bonds_of[z] = set()
        lz_pre = opens[x] + opens[y]
        for o, bl in per_nb.items():
            d = 1.0
            for b in bl:
                d *= dims[b]
                bonds_of[o].discard(b)
                del dims[b]
                del ends[b]
            lz_pre += math.log2(d)
            if chi is not None and d > chi:
                d = float(chi)
            nb = ("m", z, o)
            dims[nb] = d
            ends[nb] = [z, o]
            bonds_of[z].add(nb)
            bonds_of[o].add(nb)
        opens[z] = opens[x] + opens[y]
        del bonds_of[x]
        del bonds_of[y]
        out.append({"step": len(out), "lx": lx, "ly": ly, "lk": lk,
                    "lz": lz_pre, "lflops": lx + ly - lk + 1})
    return out


def best_of_greedy(n_tensors, bonds, open_dims=None, chi=None, seed=0,
                   first_pairs=(), trials=64, temperature=1.0):
    """Best of one deterministic and ``trials`` Boltzmann-sampled greedy paths.

    Paths are ranked by (peak log2 intermediate size, log2 total flops).
    """
    rng = np.random.default_rng(seed)
    best = None
    for t in range(trials + 1):
        temp = 0.0 if t == 0 else temperature
        s = int(rng.integers(0, 2**31))
        p = greedy_path(n_tensors, bonds, open_dims=open_dims, chi=chi, seed=s,
                        first_pairs=first_pairs, temperature=temp)
        st = path_stats(n_tensors, bonds, p, open_dims=open_dims, chi=chi)
        peak = max(max(x["lz"], x["lx"], x["ly"]) for x in st)
        tot = math.log2(sum(2.0 ** x["lflops"] for x in st))
        key = (round(peak, 6), round(tot, 6))
        if best is None or key < best[0]:
            best = (key, p)
    return best[1]
