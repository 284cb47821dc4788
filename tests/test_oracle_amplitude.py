"""Pins of the oracle's amplitudes <n|psi> (``oracle.amplitude``).

The amplitude is an entry of the ket network's coefficient tensor, which
the brute-force Koszul sum (``oracle.dense``, shared with nothing else)
gives directly. Checked on small open square lattices, for every (or a
strided subset of every) configuration, with even and with odd site
tensors and along two different paths; configurations of the wrong total
parity give exactly zero; compression with chi at least the exact bond
rank reproduces the exact amplitude.
"""

import itertools

import numpy as np
import pytest

from oracle import dense, physics as P
from oracle.amplitude import amplitude, project_first_leg, amplitude_sign
from synth import workloads as W
from synth.graphs import square_lattice
from synth.peps import make_peps, z2_leg, Z2, occupation_samples


def _kets(spec, seed):
    rng = np.random.default_rng(seed)
    return P.ket_tensors(spec, [rng.standard_normal(s.dense_shape) for s in spec.sites])


def _psi(spec, kets):
    kn = P.ket_network(spec, kets)
    return dense.koszul_value(kn.tensors, kn.bonds, list(range(spec.n_sites)))


@pytest.mark.parametrize("shape,d,stride", [((2, 2), (1, 1), 1), ((2, 3), (1, 1), 5), ((2, 2), (2, 1), 1)])
def test_amplitudes_equal_dense_coefficients(shape, d, stride):
    n, edges = square_lattice(*shape)
    spec = W.z2_peps(n, edges, *d)
    kets = _kets(spec, 40)
    psi = _psi(spec, kets)
    bonds = W.amplitude_bonds(spec)
    path = W.boundary_path(*shape)
    scale = np.abs(psi).max()
    for cfg in itertools.islice(itertools.product(range(4), repeat=n), 0, None, stride):
        m, e = amplitude(kets, bonds, cfg, path)
        assert abs(m * 2.0 ** e - psi[cfg]) <= 1e-12 * scale, cfg


@pytest.mark.parametrize("parities", [lambda s: (s % 2,), lambda s: ((s * 7 // 3) % 2,)])
def test_amplitudes_with_odd_site_tensors(parities):
    n, edges = square_lattice(2, 3)
    spec = make_peps(Z2, n, edges, phys_leg=lambda: z2_leg(2, 2, 0), bond_leg=lambda du: z2_leg(1, 1, du),
                     total_of_site=parities)
    kets = _kets(spec, 41)
    assert any(k.parity for k in kets)
    psi = _psi(spec, kets)
    bonds = W.amplitude_bonds(spec)
    scale = np.abs(psi).max()
    for path in (W.boundary_path(2, 3), [(5, 4), (6, 3), (7, 2), (8, 1), (9, 0)]):
        for cfg in itertools.islice(itertools.product(range(4), repeat=n), 0, None, 11):
            m, e = amplitude(kets, bonds, cfg, path)
            assert abs(m * 2.0 ** e - psi[cfg]) <= 1e-12 * scale, cfg


def test_wrong_parity_configurations_vanish():
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    kets = _kets(spec, 42)
    bonds = W.amplitude_bonds(spec)
    for cfg in [(2, 0, 0, 0), (2, 3, 3, 0), (1, 1, 1, 3)]:
        m, _ = amplitude(kets, bonds, cfg, W.boundary_path(2, 2))
        assert m == 0.0


def test_compressed_amplitude_with_large_chi_is_exact():
    n, edges = square_lattice(3, 3)
    spec = W.z2_peps(n, edges, 1, 1)
    kets = _kets(spec, 43)
    bonds = W.amplitude_bonds(spec)
    path = W.boundary_path(3, 3)
    for cfg in occupation_samples(n, 6, 44):
        m0, e0 = amplitude(kets, bonds, cfg, path)
        m1, e1 = amplitude(kets, bonds, cfg, path, chi=64)
        a0, a1 = m0 * 2.0 ** e0, m1 * 2.0 ** e1
        assert abs(a1 - a0) <= 1e-10 * max(abs(a0), 1e-300)


def test_projection_and_sign_helpers():
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    kets = _kets(spec, 45)
    T = kets[0]
    for idx in range(4):
        Pj = project_first_leg(T, idx)
        full = T.to_dense()
        np.testing.assert_array_equal(Pj.to_dense()[np.abs(Pj.to_dense()) > 0],
                                      full[idx][np.abs(Pj.to_dense()) > 0])
        assert Pj.parity == (T.parity ^ (idx >= 2))
    # E counts pairs of odd physical indices for even site tensors
    assert amplitude_sign(kets, (2, 3, 0, 0)) == -1.0
    assert amplitude_sign(kets, (2, 3, 2, 3)) == 1.0
    assert amplitude_sign(kets, (2, 0, 3, 0)) == -1.0


def test_boundary_path_is_a_valid_ssa_path():
    for lx, ly in [(2, 2), (3, 4), (8, 8)]:
        p = W.boundary_path(lx, ly)
        n = lx * ly
        assert len(p) == n - 1
        used = set()
        for k, (i, j) in enumerate(p):
            assert i < n + k and j < n + k and i not in used and j not in used
            used.update((i, j))
