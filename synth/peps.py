"""Leg structures of fermionic PEPS site tensors and their random entries.

A leg is described by its list of symmetry sectors (charge tuple, dimension)
in ascending charge order plus a dual flag (0 = '+', outgoing; 1 = '-',
incoming), the labels of Sec. II.A. Charges are tuples: ``(q,)`` for Z2
(q in {0, 1}) and U(1), ``(n_up, n_down)`` for U(1)xU(1).

Ket site tensors have legs ``(phys, bond to each neighbour in ascending
neighbour order)``. The physical leg is '+'. Following the default network
initialisation of Sec. IV.B (arrows point from later to earlier sites and the
'+' end is the arrow tail), the bond between sites ``i < j`` is '-' on site
``i`` and '+' on site ``j``.

Random entries are drawn as a dense array over the full leg index space
(each leg's index space is its sectors concatenated in order); the consumer
keeps only the entries its own block enumeration allows.
"""

from dataclasses import dataclass
from typing import Tuple

import numpy as np

Z2 = "Z2"
U1 = "U1"
U1U1 = "U1xU1"


@dataclass(frozen=True)
class LegSpec:
    charges: Tuple[Tuple[int, ...], ...]
    dims: Tuple[int, ...]
    dual: int

    @property
    def size(self):
        return int(sum(self.dims))


@dataclass(frozen=True)
class SiteSpec:
    legs: Tuple[LegSpec, ...]
    total: Tuple[int, ...]
    neighbours: Tuple[int, ...]   # neighbour site of bond leg 1, 2, ...

    @property
    def dense_shape(self):
        return tuple(l.size for l in self.legs)


@dataclass(frozen=True)
class PepsSpec:
    sym: str
    n_sites: int
    edges: Tuple[Tuple[int, int], ...]
    sites: Tuple[SiteSpec, ...]

    def bond_leg(self, site, nb):
        """Leg index (on ``site``) of the bond to neighbour ``nb``."""
        return 1 + self.sites[site].neighbours.index(nb)


def z2_leg(even, odd, dual):
    ch, dm = [], []
    if even:
        ch.append((0,))
        dm.append(int(even))
    if odd:
        ch.append((1,))
        dm.append(int(odd))
    return LegSpec(tuple(ch), tuple(dm), int(dual))


def u1u1_leg(sectors, dual):
    """``sectors``: mapping charge tuple -> dim; sorted lexicographically."""
    items = sorted((tuple(int(x) for x in q), int(d)) for q, d in sectors.items() if d)
    return LegSpec(tuple(q for q, _ in items), tuple(d for _, d in items), int(dual))


def make_peps(sym, n_sites, edges, phys_leg, bond_leg, total_of_site):
    """Assemble site structures on a graph.

    ``phys_leg()`` returns the physical LegSpec, ``bond_leg(dual)`` a bond
    LegSpec with the given dual, ``total_of_site(s)`` the total charge.
    """
    nbrs = [[] for _ in range(n_sites)]
    for u, v in edges:
        nbrs[u].append(v)
        nbrs[v].append(u)
    sites = []
    for s in range(n_sites):
        nb = tuple(sorted(nbrs[s]))
        legs = [phys_leg()]
        for n in nb:
            legs.append(bond_leg(1 if s < n else 0))
        sites.append(SiteSpec(tuple(legs), tuple(total_of_site(s)), nb))
    return PepsSpec(sym, n_sites, tuple(tuple(e) for e in edges), tuple(sites))


def site_values(spec: PepsSpec, site, seed, std=1.0):
    """Dense N(0, std^2) array over the full index space of one site tensor.

    Generator: ``numpy.random.default_rng([seed, site])``, row-major fill.
    """
    rng = np.random.default_rng([int(seed), int(site)])
    return rng.standard_normal(spec.sites[site].dense_shape) * float(std)


def occupation_samples(n_sites, n_samples, seed):
    """Occupation configurations with even total fermion parity.

    Physical index space per site (Z2 leg with sectors even(2), odd(2)):
    0 = |0>, 1 = |up,dn>, 2 = |up>, 3 = |dn>; indices 2, 3 are odd. Sites
    ``0..n-2`` are uniform over the 4 states; the last site is uniform over
    the 2 states that make the total parity even.
    """
    rng = np.random.default_rng(int(seed))
    out = np.empty((n_samples, n_sites), dtype=np.int64)
    for k in range(n_samples):
        cfg = rng.integers(0, 4, size=n_sites - 1)
        par = int(np.sum(cfg >= 2)) % 2
        last = int(rng.integers(0, 2))
        last = (2 + last) if par else last   # odd state fixes odd parity
        out[k, :-1] = cfg
        out[k, -1] = last
    return out
