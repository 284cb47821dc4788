"""Two-site Hubbard terms as dense 4-leg arrays (inputs to a network).

Eq. (fermi-hubbard-ham): H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i
n_i,up n_i,dn. A term acting on sites u < v is given as the dense array
G[a, b, c, d] over the physical index spaces of the legs (out_u, out_v,
in_v, in_u): G[a, b, c, d] = <a_u b_v| h |d_u c_v>, where
|x_u y_v> = (c+_u)^x (c+_v)^y |0> with modes ordered (u_up, u_dn, v_up,
v_dn) and a site state's creation string ordered up before down.

Physical index of a site: for the Z2 leg (sectors even(2), odd(2)):
0 = |0>, 1 = |up dn>, 2 = |up>, 3 = |dn>; for the U(1)xU(1) leg (sectors
(0,0), (0,1), (1,0), (1,1)): 0 = |0>, 1 = |dn>, 2 = |up>, 3 = |up dn>.
"""

import numpy as np

OCCUPATIONS = {
    "Z2": [(0, 0), (1, 1), (1, 0), (0, 1)],
    "U1xU1": [(0, 0), (0, 1), (1, 0), (1, 1)],
}


def _creation(n_modes):
    """Jordan-Wigner creation matrices, basis index = sum_m n_m 2^(n-1-m)."""
    dim = 2 ** n_modes
    ops = []
    for m in range(n_modes):
        c = np.zeros((dim, dim))
        for s in range(dim):
            occ = [(s >> (n_modes - 1 - k)) & 1 for k in range(n_modes)]
            if occ[m]:
                continue
            sign = (-1) ** sum(occ[:m])
            t = s | (1 << (n_modes - 1 - m))
            c[t, s] = sign
        ops.append(c)
    return ops


def two_site_matrix(kind, t=1.0, U=8.0):
    cd = _creation(4)
    c = [x.T for x in cd]
    if kind == "hop":
        h = np.zeros((16, 16))
        for s in range(2):
            hop = cd[s] @ c[2 + s]
            h -= t * (hop + hop.T)
        return h
    if kind == "onsite_u_first":
        return U * (cd[0] @ c[0]) @ (cd[1] @ c[1])
    if kind == "onsite_u_second":
        return U * (cd[2] @ c[2]) @ (cd[3] @ c[3])
    raise ValueError(kind)


def operator_dense(kind, sym="Z2", t=1.0, U=8.0):
    h = two_site_matrix(kind, t=t, U=U)
    occ = OCCUPATIONS[sym]

    def idx(x, y):
        bits = list(occ[x]) + list(occ[y])
        return int(sum(b << (3 - k) for k, b in enumerate(bits)))

    G = np.zeros((4, 4, 4, 4))
    for a in range(4):
        for b in range(4):
            for cc in range(4):
                for d in range(4):
                    G[a, b, cc, d] = h[idx(a, b), idx(d, cc)]
    return G
