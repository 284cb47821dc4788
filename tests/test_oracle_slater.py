"""Free-fermion pin of the oracle's amplitudes: Slater determinant fPEPS.

A Slater determinant has the closed-form coefficients
<n|psi> = det Phi[occupied modes ascending, :] (``tests.helpers``). Its
Jordan-Wigner coefficients are a plain chain product over the sites in mode
order (``synth.slater``); laid along a row snake of a square lattice (other
lattice bonds of dimension one) and turned into fermionic site tensors by
the oracle's own fermionic transposition (legs (left, phys, right) ->
(phys, neighbours ascending), Eq. transposition), the ket network must
reproduce the determinant for every configuration:

* on 2x2 and 2x3 lattices for all configurations, through the brute-force
  Koszul sum of the coefficient tensor (no amplitude machinery involved),
  which ties the construction to the closed form;
* on 3x3 (exact), 4x4 and 6x6 lattices through ``oracle.amplitude`` (projection, the
  sign of fixing the physical legs, network contraction along the
  row-by-row boundary path, exact and with chi at the bond dimension), for
  sampled configurations of the right and of the wrong particle numbers.
"""

import numpy as np
import pytest

from oracle import dense, physics as OP, symmetry as S
from oracle.amplitude import amplitude
from oracle.ops import ftranspose
from oracle.tensor import FTensor
from synth import slater as SL
from synth import workloads as W
from tests.helpers import slater_amplitude, slater_sites


def slater_network(lx, ly, phi):
    """Ket site tensors (legs: phys, neighbours ascending) and bonds."""
    sites, bonds, label = slater_sites(lx, ly, phi)
    kets = [ftranspose(FTensor.from_dense(S.Z2, legs, total, arr), perm) for legs, total, arr, perm in sites]
    return kets, bonds, label


def snake_boundary_path(lx, ly, label):
    """The row-by-row boundary path with site ids mapped to snake labels."""
    n = lx * ly
    return [tuple(int(label[t]) if t < n else t for t in step) for step in W.boundary_path(lx, ly)]


@pytest.mark.parametrize("shape,m_up,m_dn", [((2, 2), 1, 1), ((2, 2), 2, 0), ((2, 3), 2, 1), ((2, 3), 1, 2)])
def test_dense_coefficients_are_the_determinant(shape, m_up, m_dn):
    lx, ly = shape
    n = lx * ly
    phi = SL.orbitals(n, m_up, m_dn, seed=120 + 10 * n + m_up)
    kets, bonds, _ = slater_network(lx, ly, phi)
    psi = dense.koszul_value(dict(enumerate(kets)), bonds, list(range(n)))
    assert psi.shape == (4,) * n
    nonzero = 0
    for cfg in np.ndindex(*psi.shape):
        ref = slater_amplitude(phi, cfg)
        assert abs(psi[cfg] - ref) <= 1e-12 * max(1.0, abs(ref)), (cfg, psi[cfg], ref)
        nonzero += ref != 0.0
    assert nonzero > 0


def _configs(rng, n, m_up, m_dn, count):
    out = []
    for _ in range(count):
        up = rng.choice(n, m_up, replace=False)
        dn = rng.choice(n, m_dn, replace=False)
        c = np.zeros(n, dtype=np.int64)
        for i in range(n):
            u, d = i in up, i in dn
            c[i] = 1 if (u and d) else 2 if u else 3 if d else 0
        out.append(c)
    return out


@pytest.mark.parametrize("shape,m_up,m_dn,chi", [((3, 3), 2, 1, None), ((4, 4), 2, 2, 16), ((6, 6), 2, 1, 8)])
def test_amplitudes_are_the_determinant(shape, m_up, m_dn, chi):
    lx, ly = shape
    n = lx * ly
    phi = SL.orbitals(n, m_up, m_dn, seed=130 + n)
    kets, bonds, label = slater_network(lx, ly, phi)
    path = snake_boundary_path(lx, ly, label)
    rng = np.random.default_rng(131)
    cfgs = _configs(rng, n, m_up, m_dn, 12)
    # wrong particle numbers of the right parity, then of the wrong parity
    cfgs += _configs(rng, n, m_up + 1, m_dn + 1, 2) + _configs(rng, n, m_up + 1, m_dn, 2)
    refs = [slater_amplitude(phi, c) for c in cfgs]
    scale = max(abs(r) for r in refs)
    for c, ref in zip(cfgs, refs):
        mant, e = amplitude(kets, bonds, c, path, chi=chi)
        got = mant * 2.0 ** e
        assert abs(got - ref) <= 1e-12 * scale, (c, got, ref)
        if ref == 0.0 and chi is None:
            assert got == 0.0                      # structural zero, no rounding
