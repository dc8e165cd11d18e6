"""Pins of the observable oracle (charge and field profiles, surface
density, pinned static charges) against Gauss's law, closed forms, hand
examples and the agreement of the two ED formulations."""

import numpy as np
import pytest

from oracle import observables as obs
from oracle.ed import DressedED, OriginalED
from oracle.hamiltonian import Couplings, Hamiltonian
from oracle.lattice import Lattice

CPL = Couplings(t=1.0, m=0.7, g2e=1.3, g2m=0.9)


def _ground(ed, unique=True):
    e, v, gap = obs.ed_ground_state(ed)
    if unique:
        assert gap > 1e-6, "degenerate ground state: expectations not unique"
    return e, v, gap


@pytest.mark.parametrize("L,bc,Q", [((2, 2, 1), "zero_flux", 0), ((2, 1, 1), "free_flux", 1),
                                    ((2, 1, 1), "free_flux", -1), ((2, 2, 2), "zero_flux", 0)])
def test_fluxes_obey_gauss_and_agree_between_formulations(L, bc, Q):
    lat = Lattice(*L, boundary=bc)
    oe = OriginalED(lat, CPL, Q=Q)
    # conserved dangling fluxes make free-flux ground states degenerate;
    # Gauss's law holds for every state of the manifold
    e0, v, gap = _ground(oe, unique=bc == "zero_flux")
    charge, flux = obs.ed_local_expectations(oe, v)
    # Gauss's law on every site, and the total charge
    assert np.abs(flux.sum(axis=1) - charge).max() < 1e-12
    assert abs(charge.sum() - Q) < 1e-12
    # zero-flux boundary half-links carry no field
    for s in range(lat.nsites):
        for h, pres in enumerate(lat.present(s)):
            if not pres and bc == "zero_flux":
                assert flux[s, h] == 0.0
    de = DressedED(Hamiltonian(lat, CPL), Q=Q)
    e1, w, _ = _ground(de, unique=False)
    assert abs(e1 - e0) < 1e-11
    c2, f2 = obs.dressed_local_expectations(de, w)
    assert np.abs(f2.sum(axis=1) - c2).max() < 1e-12
    if gap < 1e-6:
        return
    assert np.abs(c2 - charge).max() < 1e-10
    assert np.abs(f2 - flux).max() < 1e-10


def test_plane_profiles_single_link_hand_example():
    # one link of field e from site (1,0,0) to (2,0,0) on a 4x2x1 lattice
    dims, e = (4, 2, 1), 0.3
    n = 8
    charge, flux = np.zeros(n), np.zeros((n, 6))
    x, y = 1, 2
    flux[x, 3] = e
    flux[y, 0] = -e
    charge[x], charge[y] = e, -e
    qc, ec = obs.plane_profiles(dims, charge, flux, 0)
    A = 2
    assert np.allclose(qc, [0, 2 * e / A, -2 * e / A, 0], atol=0, rtol=0)
    assert np.allclose(ec, [0, 0, 2 * e / A, 0, 0], atol=0, rtol=0)
    # along y the same link is transverse: no flux crosses a y plane
    qy, ey = obs.plane_profiles(dims, charge, flux, 1)
    assert np.array_equal(ey, np.zeros(3))
    assert np.array_equal(qy, np.zeros(2))


@pytest.mark.parametrize("dims,axis", [((4, 4, 2), 0), ((4, 4, 2), 1), ((4, 4, 2), 2), ((8, 2, 2), 0)])
def test_plane_gauss_relation_random_fields(dims, axis):
    """Any link fields on a zero-flux lattice: E^c(d+1) - E^c(d) = q_c(d)."""
    lat = Lattice(*dims)
    rng = np.random.default_rng(7)
    n = lat.nsites
    flux = np.zeros((n, 6))
    for (x, mu, y) in lat.links():
        e = rng.uniform(-1, 1)
        flux[x, 3 + mu] += e
        flux[y, mu] -= e
    charge = flux.sum(axis=1)
    qc, ec = obs.plane_profiles(dims, charge, flux, axis)
    assert ec[0] == 0.0 and abs(ec[-1]) == 0.0
    assert np.abs(np.diff(ec) - qc).max() < 1e-14


@pytest.mark.parametrize("axis", [0, 1])
def test_plane_profiles_with_dangling_faces(axis):
    """Free flux: the face terms equal the dangling fluxes along the axis,
    and Gauss's law closes with the transverse dangling flux of each plane."""
    lat = Lattice(2, 1, 1, boundary="free_flux")
    # transverse dangling fluxes fixed at 0: the charge's field leaves
    # through the two x faces
    fix = {(s, h): 0 for s in range(2) for h in (1, 2, 4, 5)}
    oe = OriginalED(lat, CPL, Q=1, dangling=fix)
    _, v, _ = _ground(oe, unique=False)
    charge, flux = obs.ed_local_expectations(oe, v)
    qc, ec = obs.plane_profiles(lat.L, charge, flux, axis)
    La = lat.L[axis]
    A = lat.nsites // La
    trans = np.zeros(La)
    face = 0.0
    for s in range(lat.nsites):
        d = lat.coords(s)[axis]
        trans[d] += sum(flux[s, h] for h in range(6) if h % 3 != axis)
        if d == 0:
            face += flux[s, axis]
    assert np.abs(np.diff(ec) - qc + 2.0 * trans / A).max() < 1e-12
    assert abs(ec[0] + 2.0 * face / A) < 1e-12
    if axis == 0:
        # all of the charge's field leaves through the two x faces
        assert abs(ec[-1] - ec[0] - 2.0 * 1 / A) < 1e-12
        assert abs(ec[0]) + abs(ec[-1]) > 1.0


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8])
def test_shell_counts_closed_form(L):
    dims = (L, L, L)
    shells = np.array([obs.shell_of(dims, s) for s in range(L ** 3)])
    for l in range(1, (L + 1) // 2 + 1):
        outer = L - 2 * (l - 1)
        inner = max(L - 2 * l, 0)
        assert np.sum(shells == l) == outer ** 3 - inner ** 3
    assert shells.max() == (L + 1) // 2


def test_surface_density_hand_example_and_sum_rule():
    dims = (4, 4, 4)
    rng = np.random.default_rng(5)
    charge = rng.uniform(-1, 1, 64)
    sig = obs.surface_density(dims, charge)
    assert sig.shape == (2,)
    # the 8 inner sites of a 4x4x4 cube form shell 2
    inner = [s for s in range(64) if all(1 <= c <= 2 for c in (s % 4, (s // 4) % 4, s // 16))]
    assert abs(sig[1] - charge[inner].mean()) < 1e-15
    # sum rule: sum_l |A(l)| sigma(l) = total charge
    assert abs(56 * sig[0] + 8 * sig[1] - charge.sum()) < 1e-13


def test_pinning_rejects_wrong_parity():
    with pytest.raises(ValueError):
        obs.pinning_potentials((4, 1, 1), {1: +1}, 10.0)
    with pytest.raises(ValueError):
        obs.pinning_potentials((4, 1, 1), {0: -1}, 10.0)
    mu = obs.pinning_potentials((4, 1, 1), {0: 1, 1: -1, 2: 0, 3: 0}, 5.0)
    assert list(mu) == [-5.0, 5.0, 5.0, -5.0]


@pytest.mark.parametrize("r", [1, 3, 5])
def test_static_potential_strong_coupling_closed_form(r):
    """t = 0, g_m = 0 on a line: two pinned opposite charges at distance r
    joined by a unit string cost V(r) = 2m + (g_e^2/2) r - lambda over the
    vacuum (linear confinement)."""
    m, g2e, lam = 2.0, 1.0, 10.0
    dims = (8, 1, 1)
    lat = Lattice(*dims)
    a, b = 2, 2 + r
    mu = obs.pinning_potentials(dims, {a: +1, b: -1}, lam)
    e_r = OriginalED(lat, Couplings(t=0.0, m=m, g2e=g2e, g2m=0.0, mu=tuple(mu))).spectrum()[0]
    e_0 = OriginalED(lat, Couplings(t=0.0, m=m, g2e=g2e, g2m=0.0)).spectrum()[0]
    assert abs((e_r - e_0) - (2 * m + 0.5 * g2e * r - lam)) < 1e-12


def test_pinned_pair_profiles_show_the_string():
    """With hopping on, the pinned pair keeps its charges and the field
    between them points from + to -."""
    dims = (8, 1, 1)
    lat = Lattice(*dims)
    mu = obs.pinning_potentials(dims, {2: +1, 5: -1}, 20.0)
    oe = OriginalED(lat, Couplings(t=0.5, m=2.0, g2e=1.0, g2m=0.0, mu=tuple(mu)))
    _, v, _ = _ground(oe)
    charge, flux = obs.ed_local_expectations(oe, v)
    qc, ec = obs.plane_profiles(dims, charge, flux, 0)
    assert qc[2] > 1.9 and qc[5] < -1.9
    assert np.all(ec[3:6] > 1.5) and np.all(np.abs(ec[:2]) < 0.2)
    assert np.abs(np.diff(ec) - qc).max() < 1e-12
