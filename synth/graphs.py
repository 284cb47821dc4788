"""Seeded graph generators for the lattices the paper studies.

Every function returns ``(n_sites, edges)`` with ``edges`` a sorted list of
``(u, v)`` pairs, ``u < v``. The generators use only ``numpy.random`` with an
explicit seed, so the instances do not depend on any graph library version.
"""

import numpy as np


def square_lattice(lx, ly):
    """Open-boundary ``lx`` x ``ly`` square lattice, sites numbered row-major."""
    edges = []
    for x in range(lx):
        for y in range(ly):
            s = x * ly + y
            if y + 1 < ly:
                edges.append((s, s + 1))
            if x + 1 < lx:
                edges.append((s, s + ly))
    return lx * ly, sorted(edges)


def random_regular_graph(degree, n, seed, max_tries=10000):
    """Random ``degree``-regular simple connected graph on ``n`` vertices.

    Configuration (pairing) model with rejection of self-loops, multi-edges
    and disconnected results, driven by ``numpy.random.default_rng(seed)``.
    The random 3-regular graphs of the paper's Sec. V.B are of this kind.
    """
    if (degree * n) % 2:
        raise ValueError("degree * n must be even")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n), degree)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if not ok:
            continue
        if not _connected(n, seen):
            continue
        return n, sorted(seen)
    raise RuntimeError("no simple connected regular graph found")


def _connected(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    stack = [0]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return len(seen) == n


def diamond_lattice(lx, ly, lz):
    """Finite diamond lattice of ``lx*ly*lz`` primitive cells (Sec. V.A).

    Primitive FCC vectors a1=(0,1,1)/2, a2=(1,0,1)/2, a3=(1,1,0)/2 with a
    two-site basis: sublattice A at the cell origin, B at (1,1,1)/4. Site
    index ``2*cell + sublattice``, cell = ``(x*ly + y)*lz + z``. Each B site
    bonds to the A sites of its own cell and of the cells shifted by +a1,
    +a2, +a3 (open boundary), giving bulk coordination 4.
    """
    def cell(x, y, z):
        return (x * ly + y) * lz + z

    edges = []
    for x in range(lx):
        for y in range(ly):
            for z in range(lz):
                b = 2 * cell(x, y, z) + 1
                for dx, dy, dz in ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    X, Y, Z = x + dx, y + dy, z + dz
                    if X < lx and Y < ly and Z < lz:
                        a = 2 * cell(X, Y, Z)
                        edges.append((min(a, b), max(a, b)))
    return 2 * lx * ly * lz, sorted(edges)
