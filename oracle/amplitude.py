"""Amplitudes <n|psi> of a fermionic PEPS (test infrastructure).

The ket network with open physical legs is the coefficient tensor Psi_n of
|psi> = sum_n Psi_n prod_i (c+_i)^{n_i} |0>, with the physical legs (leg 0
of every site tensor) in site order and the site order as the global order
(Sec. II.D). Fixing every physical index turns each site tensor T_i into
its projection T_i^{n_i} (entries T_i[n_i, ...], total charge reduced by the
charge of n_i), and the network of projections is closed.

Sign. In the global convention the value with open legs brings the open
legs to the front in order (Eq. fermionictn with the Koszul rule of Eq.
transposition). The physical leg of site i passes the bond legs of sites
j < i, whose parity in any nonzero term is p(T_j) + p(n_j). Hence

    Psi_n = (-1)^E F(T_0^{n_0} T_1^{n_1} ...),
    E = sum_i p(n_i) sum_{j<i} (p(T_j) + p(n_j))  (mod 2),

and F of the projected network is contracted with ``network`` (local
convention, dummy legs ranked by site order) along any path, exactly or with
compression as early as possible (Sec. III).
"""

from . import symmetry as S
from .tensor import FTensor
from .network import Network, network_value


def project_first_leg(T, index):
    """T^{index}: entries T[index, ...] as a tensor on the remaining legs."""
    sym = T.sym
    l0 = T.legs[0]
    off = 0
    for k, d in enumerate(l0.dims):
        if index < off + d:
            sect, loc = k, index - off
            break
        off += d
    else:
        raise ValueError("physical index out of range")
    q = S.signed(sym, l0.dual, l0.charges[sect])
    out = FTensor(sym, T.legs[1:], S.add(sym, T.total, S.neg(sym, q)))
    for key in T.keys():
        if key[0] == sect:
            out.blocks[key[1:]] = T.block(key)[loc].clone()
    return out


def index_parity(T, index):
    l0 = T.legs[0]
    off = 0
    for k, d in enumerate(l0.dims):
        if index < off + d:
            return S.parity(T.sym, l0.charges[k])
        off += d
    raise ValueError("physical index out of range")


def amplitude_sign(kets, config):
    """(-1)^E of the module docstring."""
    e, acc = 0, 0
    for T, n in zip(kets, config):
        pn = index_parity(T, int(n))
        e ^= pn & acc
        acc ^= (T.parity ^ pn)
    return -1.0 if e else 1.0


def amplitude_network(kets, bonds, config):
    """Closed network of the projections; bonds given in site-tensor legs."""
    proj = [project_first_leg(T, int(n)) for T, n in zip(kets, config)]
    b = [(t1, l1 - 1, t2, l2 - 1) for (t1, l1, t2, l2) in bonds]
    return Network(proj, b, conv="local", positions=list(range(len(kets))))


def amplitude(kets, bonds, config, path, chi=None):
    """<n|psi> as (mantissa, exp2)."""
    m, e = network_value(amplitude_network(kets, bonds, config), path, chi=chi)
    return amplitude_sign(kets, config) * m, e
