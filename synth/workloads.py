"""The seeded synthetic workloads (geometries, leg structures, seeds, paths).

Five workloads stand in for the paper's SU-optimised PEPS on the square
lattice, random 3-regular graphs (Sec. V.B) and the diamond lattice (Sec.
V.A), whose optimised weights are not available:

* ``c1``: Z2 fPEPS on a 2x3 open square lattice, phys (2|2), bond (1|1),
  exact norm <psi|psi>.
* ``c2``: Z2 fPEPS on a random 3-regular graph with 40 sites, phys (2|2),
  bond (2|2), approximate norm and one hopping term at chi = 64.
* ``c3``: U(1)xU(1) fPEPS on a 4x4x2-cell diamond cluster (64 sites), bond
  (0,0):4, (+-1,0):1, (0,+-1):1, chi = 128.
* ``c4``: Z2 fPEPS on an 8x8 square lattice, bond (3|3), 4096 sampled
  amplitudes, boundary MPS chi = 36.
* ``c5``: Z2 fPEPS on a 6x6 square lattice, bond (2|2), energy gradient,
  chi = 32.

Tensor ids of a norm network (shared by both sides so that one path serves
both): bra of site i is ``i``, ket of site i is ``n + i``, the optional
two-site operator is ``2n``. Global positions follow Fig. 4(a): bra tensors
in reverse site order, then the operator, then the kets in site order.
"""

import numpy as np

from .graphs import square_lattice, random_regular_graph, diamond_lattice
from .peps import (Z2, U1U1, z2_leg, u1u1_leg, make_peps, site_values)
from .paths import greedy_path

BASE_SEED = 20241002


def seed_of(cfg_index):
    return BASE_SEED + int(cfg_index)


def z2_peps(n, edges, d_even, d_odd, phys=(2, 2)):
    return make_peps(Z2, n, edges,
                     phys_leg=lambda: z2_leg(phys[0], phys[1], 0),
                     bond_leg=lambda dual: z2_leg(d_even, d_odd, dual),
                     total_of_site=lambda s: (0,))


def u1u1_diamond(lx, ly, lz):
    n, edges = diamond_lattice(lx, ly, lz)
    phys = {(0, 0): 1, (0, 1): 1, (1, 0): 1, (1, 1): 1}
    bond = {(0, 0): 4, (1, 0): 1, (-1, 0): 1, (0, 1): 1, (0, -1): 1}
    return make_peps(U1U1, n, edges,
                     phys_leg=lambda: u1u1_leg(phys, 0),
                     bond_leg=lambda dual: u1u1_leg(bond, dual),
                     total_of_site=lambda s: (1, 1) if s % 2 == 0 else (0, 0))


def default_std(spec, site):
    """Entry scale: 1/sqrt(dense size / phys dim / 2)."""
    shape = spec.sites[site].dense_shape
    fan = float(np.prod(shape)) / shape[0] / 2.0
    return 1.0 / np.sqrt(fan)


def all_site_values(spec, seed, std=None):
    vals = []
    for s in range(spec.n_sites):
        sd = default_std(spec, s) if std is None else std
        vals.append(site_values(spec, s, seed, sd))
    return vals


def norm_network_bonds(spec, op_sites=None):
    """Bonds ``(t1, leg1, t2, leg2, dim)`` of <psi|psi> or <psi|h|psi>.

    Ket of site s is tensor ``n+s`` with the site's legs; bra of site s is
    tensor ``s`` with the same legs in reverse order (leg k of the bra is leg
    ``L-1-k`` of the ket). The operator (tensor ``2n``) has legs
    ``(out_u, out_v, in_v, in_u)`` for ``op_sites = (u, v)``.
    """
    n = spec.n_sites
    bonds = []
    L = [len(spec.sites[s].legs) for s in range(n)]

    def bra_leg(s, k):
        return L[s] - 1 - k

    for s in range(n):
        pdim = spec.sites[s].legs[0].size
        if op_sites is not None and s in op_sites:
            continue
        bonds.append((s, bra_leg(s, 0), n + s, 0, pdim))
    if op_sites is not None:
        u, v = op_sites
        op = 2 * n
        du = spec.sites[u].legs[0].size
        dv = spec.sites[v].legs[0].size
        bonds.append((u, bra_leg(u, 0), op, 0, du))
        bonds.append((v, bra_leg(v, 0), op, 1, dv))
        bonds.append((op, 2, n + v, 0, dv))
        bonds.append((op, 3, n + u, 0, du))
    for (a, b) in spec.edges:
        ka = spec.bond_leg(a, b)
        kb = spec.bond_leg(b, a)
        d = spec.sites[a].legs[ka].size
        bonds.append((a, bra_leg(a, ka), b, bra_leg(b, kb), d))
        bonds.append((n + a, ka, n + b, kb, d))
    return bonds


def norm_network_positions(n, with_op):
    """Global position of every tensor id (Fig. 4(a) ordering)."""
    pos = {}
    for s in range(n):
        pos[s] = n - 1 - s
    off = n
    if with_op:
        pos[2 * n] = n
        off = n + 1
    for s in range(n):
        pos[n + s] = off + s
    return [pos[t] for t in range(2 * n + (1 if with_op else 0))]


def norm_path(spec, chi=None, seed=0, op_sites=None, pair_layers=True):
    """Greedy SSA path for a norm network.

    With ``pair_layers`` each bra tensor is first contracted with its ket
    partner (or, at operator sites, with the operator chain), which the
    greedy search then treats as a double-layer network.
    """
    n = spec.n_sites
    nt = 2 * n + (1 if op_sites is not None else 0)
    bonds = [(t1, t2, d) for (t1, _, t2, _, d) in norm_network_bonds(spec, op_sites)]
    first = []
    if pair_layers:
        if op_sites is not None:
            u, v = op_sites
            first.append((n + u, 2 * n))
            first.append((n + v, n + u))
            first.append((u, n + u))
            first.append((v, n + u))
        for s in range(n):
            if op_sites is not None and s in op_sites:
                continue
            first.append((s, n + s))
    return greedy_path(nt, bonds, chi=chi, seed=seed, first_pairs=first)


# --- the five workloads ---------------------------------------------------

def c1():
    n, edges = square_lattice(2, 3)
    spec = z2_peps(n, edges, 1, 1)
    return dict(name="c1_z2_2x3_exact", spec=spec, seed=seed_of(1), chi=None,
                std=1.0)


def c2(n_sites=40, chi=64, d=(2, 2), graph_seed=None):
    gs = seed_of(2) if graph_seed is None else graph_seed
    n, edges = random_regular_graph(3, n_sites, gs)
    spec = z2_peps(n, edges, d[0], d[1])
    return dict(name="c2_z2_rrg%d_chi%d" % (n_sites, chi), spec=spec,
                seed=seed_of(2), chi=chi, std=None,
                op_sites=tuple(edges[0]))


def c3(cells=(4, 4, 2), chi=128):
    spec = u1u1_diamond(*cells)
    return dict(name="c3_u1u1_diamond%dx%dx%d_chi%d" % (cells + (chi,)),
                spec=spec, seed=seed_of(3), chi=chi, std=None,
                op_sites=tuple(spec.edges[0]))


def c4(lx=8, ly=8, chi=36, n_samples=4096):
    n, edges = square_lattice(lx, ly)
    spec = z2_peps(n, edges, 3, 3)
    return dict(name="c4_z2_%dx%d_amplitudes_chi%d" % (lx, ly, chi),
                spec=spec, seed=seed_of(4), chi=chi, std=None,
                n_samples=n_samples, lx=lx, ly=ly)


def c5(lx=6, ly=6, chi=32):
    n, edges = square_lattice(lx, ly)
    spec = z2_peps(n, edges, 2, 2)
    return dict(name="c5_z2_%dx%d_grad_chi%d" % (lx, ly, chi), spec=spec,
                seed=seed_of(5), chi=chi, std=1.0, lx=lx, ly=ly)


# --- amplitudes <n|psi> (projected single-layer networks) -------------------

def amplitude_bonds(spec):
    """Bonds ``(t1, leg1, t2, leg2)`` of the ket network in site-tensor legs.

    Leg 0 of every site tensor is physical; the amplitude network joins the
    bond legs (>= 1) of the site tensors, tensor id = site id.
    """
    out = []
    for (a, b) in spec.edges:
        out.append((a, spec.bond_leg(a, b), b, spec.bond_leg(b, a)))
    return out


def boundary_path(lx, ly):
    """SSA path that absorbs an ``lx`` x ``ly`` square lattice row by row.

    Sites are numbered row-major (``s = x * ly + y``). The boundary starts as
    row 0; every later row is absorbed column by column (boundary tensor y
    with site (x, y)), and the final boundary is contracted left to right.
    """
    n = lx * ly
    cur = list(range(ly))
    path = []
    nxt = n
    for x in range(1, lx):
        for y in range(ly):
            path.append((cur[y], x * ly + y))
            cur[y] = nxt
            nxt += 1
    acc = cur[0]
    for y in range(1, ly):
        path.append((acc, cur[y]))
        acc = nxt
        nxt += 1
    return path


def hubbard_terms(spec):
    """Two-site terms of the Hubbard Hamiltonian (Eq. fermi-hubbard-ham).

    ``[(kind, (u, v))]`` with u < v: a hopping term on every edge, and the
    on-site term of every site s on the pair (s, first neighbour of s),
    kind ``onsite_u_first`` when s is the smaller site of the pair and
    ``onsite_u_second`` otherwise (see ``synth.operators``).
    """
    out = [("hop", (a, b)) for (a, b) in spec.edges]
    for s in range(spec.n_sites):
        nb = spec.sites[s].neighbours[0]
        out.append(("onsite_u_first", (s, nb)) if s < nb else ("onsite_u_second", (nb, s)))
    return out


def norm_boundary_path(spec, lx, ly, op_sites=None):
    """SSA path of a norm network on an ``lx`` x ``ly`` lattice, row by row.

    Tensor ids as in ``norm_network_bonds``. Each bra is first contracted
    with its ket (the operator of a term joins the ket and then the bra of
    its first site, and stays bonded to the second site); the double-layer
    sites are then absorbed into a boundary row by row, column by column,
    and the final boundary is contracted left to right (the boundary-MPS
    order, with compression as early as possible applied by the driver).
    """
    n = lx * ly
    path = []
    nxt = 2 * n + (1 if op_sites is not None else 0)
    owner = {}
    if op_sites is not None:
        u, v = op_sites
        path.append((n + u, 2 * n))
        path.append((u, nxt))
        owner[u] = nxt + 1
        nxt += 2
    for s in range(n):
        if s in owner:
            continue
        path.append((s, n + s))
        owner[s] = nxt
        nxt += 1
    # boundary: column -> current id; ids covering several columns are
    # shared and updated together
    col = [owner[y] for y in range(ly)]
    absorbed = set(owner[y] for y in range(ly))

    def merge(a, b):
        nonlocal nxt
        path.append((a, b))
        new = nxt
        nxt += 1
        for c in range(ly):
            if col[c] in (a, b):
                col[c] = new
        return new

    for x in range(1, lx):
        for y in range(ly):
            t = owner[x * ly + y]
            if t in absorbed:
                continue
            absorbed.add(t)
            new = merge(col[y], t)
            # an operator pair spanning two columns of this row joins them
            for c in range(ly):
                if c != y and owner[x * ly + c] == t and col[c] != new:
                    merge(new, col[c])
    done = []
    for c in range(ly):
        if col[c] not in done:
            done.append(col[c])
    acc = done[0]
    for t in done[1:]:
        path.append((acc, t))
        acc = nxt
        nxt += 1
    return path


def norm_layer_path(spec, lx, ly, op_sites=None):
    """SSA path of a norm network absorbed layer by layer, row by row.

    Tensor ids as in ``norm_network_bonds``. The boundary starts as the
    kets of row 0; the bras of that row are absorbed column by column, then
    for every later row its kets and then its bras. The operator of a term
    is first contracted with the ket of its first site. Absorbing one layer
    at a time keeps the bonds that form between boundary tensors at
    chi * D (bra and ket bonds are never absorbed together), the order of
    boundary-MPS contraction with compression as early as possible.
    """
    n = lx * ly
    path = []
    nxt = 2 * n + (1 if op_sites is not None else 0)
    ket = {s: n + s for s in range(n)}
    if op_sites is not None:
        path.append((n + op_sites[0], 2 * n))
        ket[op_sites[0]] = nxt
        nxt += 1
    col = [ket[y] for y in range(ly)]

    def absorb(y, t):
        nonlocal nxt
        path.append((col[y], t))
        col[y] = nxt
        nxt += 1

    for y in range(ly):
        absorb(y, y)
    for x in range(1, lx):
        for y in range(ly):
            absorb(y, ket[x * ly + y])
        for y in range(ly):
            absorb(y, x * ly + y)
    acc = col[0]
    for t in col[1:]:
        path.append((acc, t))
        acc = nxt
        nxt += 1
    return path
