"""Jordan-Wigner Fock space, Hubbard terms and PEPS norm networks.

Conventions the paper leaves open (each is pinned by exact diagonalisation
in the tests):

* Local basis of a Z2 physical leg (sectors even(2), odd(2)): index
  0 = |0>, 1 = |up dn> = c+_up c+_dn |0>, 2 = |up>, 3 = |dn>. For a
  U(1)xU(1) leg (sectors (0,0), (0,1), (1,0), (1,1), dim 1 each): 0 = |0>,
  1 = |dn>, 2 = |up>, 3 = |up dn>.
* Modes are ordered site-major, up before down; the site order is the
  global order of the ket tensors. The ket network with open physical legs
  in site order is the coefficient tensor Psi_n of
  |psi> = sum_n Psi_n prod_i (c+_i)^{n_i} |0>.
* Bra (Sec. II.D, Fig. 4a): reverse the order of the tensors and the legs
  of every tensor, flip duals, conjugate (entries are real here).
* A two-site operator h on sites u < v is the tensor G with legs
  (out_u, out_v, in_v, in_u), duals (+, +, -, -) and entries
  G[a, b, c, d] = <a_u b_v| h |d_u c_v> in the two-site basis
  |x_u y_v> = (c+_u)^x (c+_v)^y |0>; it sits between bra and ket in the
  global order.
* Hubbard Hamiltonian, Eq. (fermi-hubbard-ham):
  H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i n_i,up n_i,dn.
"""

import numpy as np
import scipy.sparse as sp

from . import symmetry as S
from .tensor import FTensor, make_leg
from .ops import dagger
from .network import Network

# occupations (n_up, n_dn) of the physical index
OCC = {
    S.Z2: [(0, 0), (1, 1), (1, 0), (0, 1)],
    S.U1U1: [(0, 0), (0, 1), (1, 0), (1, 1)],
}


# --- Fock space -------------------------------------------------------------

def annihilators(n_modes):
    """JW annihilation operators; basis index = sum_m n_m 2^(n_modes-1-m)."""
    I = sp.identity(2, format="csr")
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    ops = []
    for m in range(n_modes):
        mats = [Z] * m + [a] + [I] * (n_modes - m - 1)
        op = mats[0]
        for x in mats[1:]:
            op = sp.kron(op, x, format="csr")
        ops.append(op.tocsr())
    return ops


def fock_index(occ_modes):
    n = len(occ_modes)
    return int(sum(int(b) << (n - 1 - m) for m, b in enumerate(occ_modes)))


def psi_to_fock(psi, sym):
    """Dense Psi over site physical indices -> Fock vector (2 modes per site)."""
    n = psi.ndim
    vec = np.zeros(2 ** (2 * n))
    occ = OCC[sym]
    for idx in np.ndindex(*psi.shape):
        modes = []
        for i in idx:
            modes += list(occ[i])
        vec[fock_index(modes)] += psi[idx]
    return vec


def hubbard(n_sites, edges, t=1.0, U=8.0):
    c = annihilators(2 * n_sites)
    H = sp.csr_matrix((2 ** (2 * n_sites),) * 2)
    for (i, j) in edges:
        for s in range(2):
            a, b = 2 * i + s, 2 * j + s
            hop = c[a].T @ c[b]
            H = H - t * (hop + hop.T)
    for i in range(n_sites):
        nu = c[2 * i].T @ c[2 * i]
        nd = c[2 * i + 1].T @ c[2 * i + 1]
        H = H + U * (nu @ nd)
    return H.tocsr()


def hopping_term(n_sites, u, v, t=1.0):
    c = annihilators(2 * n_sites)
    H = sp.csr_matrix((2 ** (2 * n_sites),) * 2)
    for s in range(2):
        hop = c[2 * u + s].T @ c[2 * v + s]
        H = H - t * (hop + hop.T)
    return H.tocsr()


def onsite_term(n_sites, u, U=8.0):
    c = annihilators(2 * n_sites)
    nu = c[2 * u].T @ c[2 * u]
    nd = c[2 * u + 1].T @ c[2 * u + 1]
    return (U * (nu @ nd)).tocsr()


# --- two-site operator tensors ---------------------------------------------

def two_site_local(kind, t=1.0, U=8.0):
    """16x16 matrix of a two-site term on modes (u_up, u_dn, v_up, v_dn)."""
    c = annihilators(4)
    if kind == "hop":
        h = sp.csr_matrix((16, 16))
        for s in range(2):
            hop = c[s].T @ c[2 + s]
            h = h - t * (hop + hop.T)
    elif kind == "onsite_u":
        h = U * (c[0].T @ c[0]) @ (c[1].T @ c[1])
    elif kind == "nn_u":
        h = (c[0].T @ c[0]) @ (c[1].T @ c[1])
    elif kind == "hubbard_bond":
        raise ValueError("use hop + onsite terms separately")
    else:
        raise ValueError(kind)
    return np.asarray(h.todense())


def operator_tensor(h16, phys_leg, sym):
    """G[a, b, c, d] = <a_u b_v| h |d_u c_v>, legs (out_u, out_v, in_v, in_u)."""
    occ = OCC[sym]
    G = np.zeros((4, 4, 4, 4))
    for a in range(4):
        for b in range(4):
            row = fock_index(list(occ[a]) + list(occ[b]))
            for cc in range(4):
                for d in range(4):
                    col = fock_index(list(occ[d]) + list(occ[cc]))
                    G[a, b, cc, d] = h16[row, col]
    out_l = make_leg(sym, phys_leg.charges, phys_leg.dims, 0)
    in_l = make_leg(sym, phys_leg.charges, phys_leg.dims, 1)
    T = FTensor.from_dense(sym, [out_l, out_l, in_l, in_l], S.zero(sym), G)
    if not np.allclose(T.to_dense(), G):
        raise ValueError("operator does not conserve the symmetry")
    return T


# --- PEPS tensors and norm networks ----------------------------------------

def leg_from_spec(sym, ls):
    return make_leg(sym, ls.charges, ls.dims, ls.dual)


def ket_tensors(spec, values):
    """FTensors of the ket sites from a synth PepsSpec and dense values."""
    sym = spec.sym
    out = []
    for s, site in enumerate(spec.sites):
        legs = [leg_from_spec(sym, l) for l in site.legs]
        out.append(FTensor.from_dense(sym, legs, site.total, values[s]))
    return out


def norm_network(spec, kets, op=None, op_sites=None, conv="global"):
    """<psi|psi> (or <psi|G|psi>) with ids bra s -> s, ket s -> n+s, op -> 2n.

    Positions follow Fig. 4(a): bras in reverse site order, the operator,
    then kets in site order. Bonds as in ``synth.workloads``.
    """
    from synth.workloads import norm_network_bonds, norm_network_positions
    n = spec.n_sites
    tensors = {}
    for s in range(n):
        tensors[s] = dagger(kets[s])
        tensors[n + s] = kets[s]
    if op is not None:
        tensors[2 * n] = op
    bonds = [(t1, l1, t2, l2) for (t1, l1, t2, l2, _) in
             norm_network_bonds(spec, op_sites if op is not None else None)]
    pos = norm_network_positions(n, op is not None)
    return Network(tensors, bonds, conv=conv, positions=pos)


def ket_network(spec, kets, conv="global"):
    """Ket tensors alone (open physical legs), positions = site order."""
    n = spec.n_sites
    bonds = []
    for (a, b) in spec.edges:
        bonds.append((a, spec.bond_leg(a, b), b, spec.bond_leg(b, a)))
    return Network({s: kets[s] for s in range(n)}, bonds, conv=conv,
                   positions=list(range(n)))
