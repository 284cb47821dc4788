"""Random structures for oracle tests (test-only helpers)."""

import itertools

import numpy as np

from oracle import symmetry as S
from oracle.tensor import FTensor, make_leg


def rand_leg(rng, sym, dual=None, maxd=2):
    if sym == S.Z2:
        ch = [(0,), (1,)]
    elif sym == S.U1:
        ch = [(-1,), (0,), (1,)]
    else:
        ch = [(0, 0), (1, 0), (0, 1), (-1, 0)]
    dims = [int(rng.integers(1, maxd + 1)) for _ in ch]
    d = int(rng.integers(0, 2)) if dual is None else dual
    return make_leg(sym, ch, dims, d)


def partner(leg):
    """Leg that can be contracted with ``leg`` (opposite dual, same sectors)."""
    from oracle.tensor import Leg
    return Leg(leg.charges, leg.dims, 1 - leg.dual)


def rand_tensor(rng, sym, legs, total=None, parity=None):
    if total is None:
        if sym == S.Z2:
            total = (int(rng.integers(0, 2)) if parity is None else parity,)
        elif sym == S.U1:
            total = (int(rng.integers(-1, 2)),) if parity is None else ((parity,))
        else:
            total = (0, 0) if parity in (None, 0) else (1, 0)
    shape = tuple(l.size for l in legs)
    arr = rng.standard_normal(shape)
    return FTensor.from_dense(sym, legs, total, arr)


def random_network(rng, sym, n_tensors, n_bonds, n_open=0, odd_frac=0.3,
                   maxd=2, connected=True):
    """Random network: tensors with random legs, bonds between random pairs."""
    legs = {t: [] for t in range(n_tensors)}
    bonds = []
    pairs = []
    if connected:
        perm = rng.permutation(n_tensors)
        for k in range(1, n_tensors):
            a = int(perm[k]); b = int(perm[int(rng.integers(0, k))])
            pairs.append((a, b))
    while len(pairs) < n_bonds:
        a, b = rng.choice(n_tensors, size=2, replace=False)
        pairs.append((int(a), int(b)))
    for (a, b) in pairs:
        la = rand_leg(rng, sym, maxd=maxd)
        lb = partner(la)
        # insert at random positions
        pa = int(rng.integers(0, len(legs[a]) + 1))
        pb = int(rng.integers(0, len(legs[b]) + 1))
        legs[a].insert(pa, ("b", len(bonds), la))
        legs[b].insert(pb, ("b", len(bonds), lb))
        bonds.append((a, b))
    for _ in range(n_open):
        a = int(rng.integers(0, n_tensors))
        pa = int(rng.integers(0, len(legs[a]) + 1))
        legs[a].insert(pa, ("o", None, rand_leg(rng, sym, maxd=maxd)))
    tensors = {}
    for t in range(n_tensors):
        par = 1 if rng.random() < odd_frac else 0
        tl = [x[2] for x in legs[t]]
        tensors[t] = rand_tensor(rng, sym, tl, parity=par)
    bl = []
    for bi in range(len(bonds)):
        ends = []
        for t in range(n_tensors):
            for li, x in enumerate(legs[t]):
                if x[0] == "b" and x[1] == bi:
                    ends.append((t, li))
        (t1, l1), (t2, l2) = ends
        bl.append((t1, l1, t2, l2))
    return tensors, bl


def random_ssa_path(rng, tensors, bonds):
    """Random SSA path contracting connected pairs (falls back to any pair)."""
    n = len(tensors)
    alive = {t: {t} for t in range(n)}
    adj = set()
    for (t1, _, t2, _) in bonds:
        adj.add((t1, t2))
        adj.add((t2, t1))
    ids = {t: t for t in range(n)}
    nxt = n
    path = []
    groups = [{t} for t in range(n)]
    gid = list(range(n))
    while len(groups) > 1:
        cand = []
        for i in range(len(groups)):
            for j in range(i + 1, len(groups)):
                if any((a, b) in adj for a in groups[i] for b in groups[j]):
                    cand.append((i, j))
        if not cand:
            cand = [(0, 1)]
        i, j = cand[int(rng.integers(0, len(cand)))]
        if rng.random() < 0.5:
            i, j = j, i
        path.append((gid[i], gid[j]))
        new = groups[i] | groups[j]
        for k in sorted((i, j), reverse=True):
            del groups[k]
            del gid[k]
        groups.append(new)
        gid.append(nxt)
        nxt += 1
    return path


def slater_amplitude(phi, config):
    """Closed form of a Slater determinant's Jordan-Wigner coefficient.

    |psi> = b+_1 ... b+_M |0> with b+_k = sum_m phi[m, k] c+_m: expanding the
    product and sorting each term's creation operators into ascending mode
    order gives <n|psi> = det phi[occupied modes ascending, :]. Modes of site
    i: 2i (up), 2i+1 (down); physical index 0 = |0>, 1 = |up,dn>, 2 = |up>,
    3 = |dn>.
    """
    modes = {0: (), 1: (0, 1), 2: (0,), 3: (1,)}
    occ = []
    for i, p in enumerate(config):
        occ += [2 * i + loc for loc in modes[int(p)]]
    if len(occ) != phi.shape[1]:
        return 0.0
    return float(np.linalg.det(phi[occ, :])) if occ else 1.0


def slater_sites(lx, ly, phi):
    """Site structures of the Slater fPEPS on a snake-labelled lattice.

    Per site: (legs in the chain layout (left, phys, right, other bonds),
    total charge, dense array, perm) where ``perm`` is the fermionic
    transposition to the PEPS layout (phys, neighbours ascending); bonds
    ``(t1, l1, t2, l2)`` in PEPS legs; the snake label of every site. Chain
    bonds carry the orbital subsets (Z2 sectors 2^(M-1) | 2^(M-1)), the
    other lattice bonds one even state; the bond between i < j is '-' on i.
    """
    from synth import slater as SL
    n, edges, label = SL.snake_square_lattice(lx, ly)
    m = phi.shape[1]
    arrs = SL.chain_arrays(phi)
    nbrs = [sorted([b for a, b in edges if a == s] + [a for a, b in edges if b == s]) for s in range(n)]
    phys = make_leg(S.Z2, [(0,), (1,)], [2, 2], 0)
    half = 1 << (m - 1)
    out = []
    for j in range(n):
        def bond(nb):
            dual = 1 if j < nb else 0
            if abs(nb - j) == 1:
                return make_leg(S.Z2, [(0,), (1,)], [half, half], dual)
            return make_leg(S.Z2, [(0,)], [1], dual)
        chain = ([j - 1] if j > 0 else []) + ([j + 1] if j < n - 1 else [])
        rungs = [nb for nb in nbrs[j] if nb not in chain]
        legs = ([bond(j - 1)] if j > 0 else []) + [phys] + ([bond(j + 1)] if j < n - 1 else [])
        legs += [bond(nb) for nb in rungs]
        arr = arrs[j].reshape(arrs[j].shape + (1,) * len(rungs))
        total = (m % 2,) if j == n - 1 else (0,)
        where, k = {}, 0
        if j > 0:
            where[j - 1] = 0
            k = 1
        pphys = k
        k += 1
        if j < n - 1:
            where[j + 1] = k
            k += 1
        for nb in rungs:
            where[nb] = k
            k += 1
        perm = [pphys] + [where[nb] for nb in nbrs[j]]
        out.append((legs, total, arr, perm))
    bonds = [(a, 1 + nbrs[a].index(b), b, 1 + nbrs[b].index(a)) for a, b in edges]
    return out, bonds, label
