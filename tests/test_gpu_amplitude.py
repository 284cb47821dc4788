"""GPU parity of the amplitudes <n|psi> (``ftn_amplitudes``) with the oracle.

Exact amplitudes (no compression) agree with the oracle to 1e-12 of the
largest amplitude (a few chained FP64 contractions of O(1) entries). The
8x8 workload (Z2, bond (3|3), boundary path, chi = 36) is compared on a
sample subset at 1e-8 relative: both sides compress every bond larger than
chi as soon as it forms, but the library reaches the kept subspace through
Gram matrices and the oracle through SVD, so directions with singular values
near the cutoff can differ at that level. Configurations of the wrong parity
give exactly zero; results do not depend on the number of workers.
"""

import itertools

import numpy as np
import pytest
import torch

from oracle import physics as OP
from oracle.amplitude import amplitude
from synth import workloads as W
from synth.graphs import square_lattice
from synth.peps import make_peps, z2_leg, Z2, occupation_samples
from tests.gpu_helpers import to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2410_02215_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    P.load_library()
    return P


def _kets(spec, seed):
    rng = np.random.default_rng(seed)
    return OP.ket_tensors(spec, [rng.standard_normal(s.dense_shape) for s in spec.sites])


def _oracle(kets, bonds, cfgs, path, chi=None):
    out = []
    for c in cfgs:
        m, e = amplitude(kets, bonds, c, path, chi=chi)
        out.append(m * 2.0 ** e)
    return np.array(out)


def _gpu(P, kets, bonds, cfgs, path, chi=0, nworkers=8):
    sites = [to_gpu(T) for T in kets]
    m, e = P.amplitudes(sites, bonds, path, cfgs, chi=chi, nworkers=nworkers)
    return m * np.exp2(e.astype(np.float64)), (m, e)


@pytest.mark.parametrize("shape,d", [((2, 2), (1, 1)), ((2, 3), (1, 1)), ((3, 3), (2, 1))])
def test_exact_amplitudes_match_oracle(P, shape, d):
    n, edges = square_lattice(*shape)
    spec = W.z2_peps(n, edges, *d)
    kets = _kets(spec, 50)
    bonds = W.amplitude_bonds(spec)
    path = W.boundary_path(*shape)
    cfgs = occupation_samples(n, 24, 51)
    ref = _oracle(kets, bonds, cfgs, path)
    got, _ = _gpu(P, kets, bonds, cfgs, path)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_odd_site_tensors_and_other_paths(P):
    n, edges = square_lattice(2, 3)
    spec = make_peps(Z2, n, edges, phys_leg=lambda: z2_leg(2, 2, 0), bond_leg=lambda du: z2_leg(1, 1, du),
                     total_of_site=lambda s: ((s * 7 // 3) % 2,))
    kets = _kets(spec, 52)
    bonds = W.amplitude_bonds(spec)
    cfgs = np.array(list(itertools.islice(itertools.product(range(4), repeat=n), 0, None, 37)))
    for path in (W.boundary_path(2, 3), [(5, 4), (6, 3), (7, 2), (8, 1), (9, 0)]):
        ref = _oracle(kets, bonds, cfgs, path)
        got, _ = _gpu(P, kets, bonds, cfgs, path, nworkers=3)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_wrong_parity_gives_zero(P):
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    kets = _kets(spec, 53)
    got, (m, e) = _gpu(P, kets, W.amplitude_bonds(spec), [(2, 0, 0, 0), (1, 1, 3, 0)], W.boundary_path(2, 2))
    assert np.all(m == 0.0)


def test_full_size_8x8_chi36_subset(P):
    cfg = W.c4()
    spec = cfg["spec"]
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    bonds = W.amplitude_bonds(spec)
    path = W.boundary_path(cfg["lx"], cfg["ly"])
    cfgs = occupation_samples(spec.n_sites, 6, cfg["seed"] + 1)
    got, (m, e) = _gpu(P, kets, bonds, cfgs, path, chi=cfg["chi"])
    for k, c in enumerate(cfgs):
        rm, re_ = amplitude(kets, bonds, c, path, chi=cfg["chi"])
        # compare mantissas on a common exponent (the values are ~2^-150)
        a = m[k] * 2.0 ** (int(e[k]) - re_)
        assert abs(a - rm) <= 1e-8 * abs(rm), (k, a, rm)


def test_worker_count_does_not_change_results(P):
    n, edges = square_lattice(3, 3)
    spec = W.z2_peps(n, edges, 2, 2)
    kets = _kets(spec, 54)
    bonds = W.amplitude_bonds(spec)
    path = W.boundary_path(3, 3)
    cfgs = occupation_samples(n, 40, 55)
    _, (m1, e1) = _gpu(P, kets, bonds, cfgs, path, chi=6, nworkers=1)
    _, (m8, e8) = _gpu(P, kets, bonds, cfgs, path, chi=6, nworkers=8)
    np.testing.assert_array_equal(m1, m8)
    np.testing.assert_array_equal(e1, e8)


def test_bad_arguments_are_reported(P):
    n, edges = square_lattice(2, 2)
    spec = W.z2_peps(n, edges, 1, 1)
    kets = _kets(spec, 56)
    sites = [to_gpu(T) for T in kets]
    bonds = W.amplitude_bonds(spec)
    with pytest.raises(P.FtnError) as e:
        P.amplitudes(sites, bonds, W.boundary_path(2, 2), [(0, 0, 0, 4)])
    assert e.value.code == -1
    with pytest.raises(P.FtnError) as e:
        P.amplitudes(sites, [(0, 0, 1, 1)] + bonds[1:], W.boundary_path(2, 2), [(0, 0, 0, 0)])
    assert e.value.code == -1


@pytest.mark.parametrize("shape,m_up,m_dn,chi", [((4, 4), 2, 2, 16), ((6, 6), 2, 1, 8), ((8, 8), 2, 2, 36)])
def test_slater_amplitudes_are_the_determinant(P, shape, m_up, m_dn, chi):
    # free-fermion fPEPS (a Slater determinant laid along a row snake, the
    # chain bonds 2^M wide): the library's amplitudes against the closed form
    # det Phi[occupied modes, :], with chi at or above the bond dimension;
    # site tensors are built in the chain layout and brought to the PEPS
    # layout by the library's own fermionic transposition
    from synth import slater as SL
    from tests.gpu_helpers import legs_abi
    from tests.helpers import slater_amplitude, slater_sites
    lx, ly = shape
    n = lx * ly
    phi = SL.orbitals(n, m_up, m_dn, seed=130 + n)
    sites, bonds, label = slater_sites(lx, ly, phi)
    gsites = []
    for legs, total, arr, perm in sites:
        dense = torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=torch.float64)
        T = P.Tensor.from_dense(0, legs_abi(legs), (total[0], 0), dense)
        gsites.append(P.ftranspose(T, perm))
    path = [tuple(int(label[t]) if t < n else t for t in step) for step in W.boundary_path(lx, ly)]
    rng = np.random.default_rng(131)
    cfgs = []
    for mu, md, cnt in ((m_up, m_dn, 24), (m_up + 1, m_dn + 1, 2), (m_up + 1, m_dn, 2)):
        for _ in range(cnt):
            up = set(rng.choice(n, mu, replace=False).tolist())
            dn = set(rng.choice(n, md, replace=False).tolist())
            cfgs.append([1 if (i in up and i in dn) else 2 if i in up else 3 if i in dn else 0 for i in range(n)])
    cfgs = np.array(cfgs)
    refs = np.array([slater_amplitude(phi, c) for c in cfgs])
    m, e = P.amplitudes(gsites, bonds, path, cfgs, chi=chi, nworkers=4)
    got = m * np.exp2(e.astype(np.float64))
    scale = np.abs(refs).max()
    err = np.abs(got - refs).max() / scale
    print("slater %dx%d M=%d+%d chi=%d: max error %.3g of the largest amplitude" % (lx, ly, m_up, m_dn, chi, err))
    # the bonds are compressed wherever they exceed chi (every cut of the
    # state has rank at most 2^M <= chi, so only zero directions are cut)
    assert err <= 1e-12, err
    # wrong parity: exactly zero
    assert np.all(got[-2:] == 0.0)
