"""Inputs of the free-fermion (Slater determinant) fPEPS checks.

A Slater determinant |psi> = b+_1 ... b+_M |0>, b+_k = sum_m Phi[m, k] c+_m,
has the Jordan-Wigner coefficients

    <n|psi> = det Phi[occupied modes of n in ascending order, :]

(expand the product of the b+_k and sort each term's creation operators:
the sign of the sorting permutation is the determinant's). Modes are
numbered site-major, up before down: mode 2i is (i, up), mode 2i+1 is
(i, down), the order of the physical basis 0 = |0>, 1 = |up,dn> =
c+_up c+_dn |0>, 2 = |up>, 3 = |dn>.

Sweeping the modes in that order, the coefficient is a product of
transfer matrices over the set U of orbitals already used: an occupied mode
m takes an unused orbital k with the factor Phi[m, k] times (-1)^(number of
used orbitals above k), the inversions it adds to the assignment of
orbitals to ascending modes. This module only builds those per-site arrays
(plain numbers: a chain A_0 A_1 ... A_{N-1} whose ordinary matrix product is
the coefficient) and the lattice they are laid on; turning them into
fermionic site tensors (the leg order of a PEPS site) is left to the
consumer's own fermionic transposition.

Bond index space of a chain bond: the 2^M subsets U of the M orbitals as
bitmasks, even-size subsets first, then odd-size ones, each group in
ascending bitmask order (a Z2 leg with sectors (2^(M-1) | 2^(M-1))).
"""

import numpy as np


def snake_square_lattice(lx, ly):
    """Open ``lx`` x ``ly`` square lattice labelled along a row snake.

    Row x is visited left to right for even x and right to left for odd x,
    so consecutive labels are always neighbours (a Hamiltonian path).
    Returns ``(n, edges, label)`` with ``label[x * ly + y]`` the snake label
    of site (x, y) and edges in snake labels, ``u < v``, sorted.
    """
    label = np.zeros(lx * ly, dtype=np.int64)
    t = 0
    for x in range(lx):
        cols = range(ly) if x % 2 == 0 else range(ly - 1, -1, -1)
        for y in cols:
            label[x * ly + y] = t
            t += 1
    edges = []
    for x in range(lx):
        for y in range(ly):
            s = label[x * ly + y]
            if y + 1 < ly:
                u = label[x * ly + y + 1]
                edges.append((int(min(s, u)), int(max(s, u))))
            if x + 1 < lx:
                u = label[(x + 1) * ly + y]
                edges.append((int(min(s, u)), int(max(s, u))))
    return lx * ly, sorted(edges), label


def subset_order(m):
    """Bitmasks of the bond index space in order (even sizes, then odd)."""
    even = [u for u in range(1 << m) if bin(u).count("1") % 2 == 0]
    odd = [u for u in range(1 << m) if bin(u).count("1") % 2 == 1]
    return even + odd


def orbitals(n_sites, m_up, m_dn, seed):
    """Phi (2N x (m_up + m_dn)): up orbitals live on up modes, down on down.

    Entries N(0, 1) from ``numpy.random.default_rng(seed)``.
    """
    rng = np.random.default_rng(int(seed))
    phi = np.zeros((2 * n_sites, m_up + m_dn))
    phi[0::2, :m_up] = rng.standard_normal((n_sites, m_up))
    phi[1::2, m_up:] = rng.standard_normal((n_sites, m_dn))
    return phi


# modes occupied by each physical index, in mode order (up = 0, down = 1)
PHYS_MODES = {0: (), 1: (0, 1), 2: (0,), 3: (1,)}


def chain_arrays(phi):
    """Arrays A_j of the chain, j = 0 .. N-1.

    A_0 has axes (phys, right), A_{N-1} (left, phys), the others
    (left, phys, right); the left index of A_0 is the empty set and the
    right index of A_{N-1} the full set, both dropped.
    """
    nm, m = phi.shape
    n = nm // 2
    order = subset_order(m)
    pos = {u: i for i, u in enumerate(order)}
    full = (1 << m) - 1
    out = []
    for j in range(n):
        A = np.zeros((1 << m, 4, 1 << m))
        for U in range(1 << m):
            for p, modes in PHYS_MODES.items():
                # every way of giving the occupied modes distinct unused orbitals
                states = [(U, 1.0)]
                for loc in modes:
                    mode = 2 * j + loc
                    nxt = []
                    for (V, c) in states:
                        for k in range(m):
                            if V >> k & 1 or phi[mode, k] == 0.0:
                                continue
                            above = bin(V >> (k + 1)).count("1")
                            nxt.append((V | 1 << k, c * phi[mode, k] * (-1.0) ** above))
                    states = nxt
                for (V, c) in states:
                    A[pos[U], p, pos[V]] += c
        if j == 0:
            A = A[pos[0]]                 # (phys, right)
        if j == n - 1:
            A = A[..., pos[full]]         # (left, phys) or (phys,) for n == 1
        out.append(A)
    return out

