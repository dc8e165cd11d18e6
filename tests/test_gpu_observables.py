"""GPU parity of the observable suite: site charges and fluxes, plane
profiles, surface density and pinned static charges from the HIP sweep,
against the oracle's profiles of the exact ground state (original-
formulation ED) on lattices where the bond dimension is exact, and
against Gauss's law at sizes ED cannot reach."""

import numpy as np
import pytest

from oracle import observables as obs
from oracle.ed import OriginalED
from oracle.hamiltonian import Couplings
from oracle.lattice import Lattice
from paper_2011_10658_amd import lib

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CPL = Couplings(t=1.0, m=0.7, g2e=1.3, g2m=0.9)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = lib.Context(0)
    yield c
    c.close()


def run(ctx, L, bc, cpl, chi, pins=None, lam=0.0, Q=0, sweeps=3, seed=11):
    ctx.set_lattice(*L, bc)
    ctx.set_couplings(cpl.t, cpl.m, cpl.g2e, cpl.g2m)
    if pins:
        ctx.pin_charges(pins, lam)
    ctx.set_charge_sector(Q)
    ctx.set_bond_dim(chi)
    ctx.set_penalty(20.0, 0, 0)
    ctx.set_lanczos(40, 3, 1e-13)
    ctx.set_precision(lib.FP64)
    ctx.build_hamiltonian()
    ctx.init_state(seed)
    return ctx.sweep(sweeps)[-1]["energy"]


def ed_reference(L, cpl, pins=None, lam=0.0, Q=0, boundary="zero_flux"):
    lat = Lattice(*L, boundary=boundary)
    if pins:
        mu = obs.pinning_potentials(L, pins, lam)
        cpl = Couplings(t=cpl.t, m=cpl.m, g2e=cpl.g2e, g2m=cpl.g2m, mu=tuple(mu))
    ed = OriginalED(lat, cpl, Q=Q)
    e0, v, gap = obs.ed_ground_state(ed)
    assert gap > 1e-6
    return e0, obs.ed_local_expectations(ed, v)


CASES = [
    ((2, 2, 1), CPL, None, 0.0, 64),
    ((4, 1, 1), CPL, None, 0.0, 64),
    # pinned pair at distance 3 on a line (confinement set-up)
    ((8, 1, 1), Couplings(t=0.5, m=2.0, g2e=1.0, g2m=0.0), {2: +1, 5: -1}, 20.0, 64),
    # capacitor plates on the two x faces of a 4x2x1 lattice
    ((4, 2, 1), Couplings(t=1.0, m=1.0, g2e=1.0, g2m=1.0), {0: +1, 4: 0, 3: -1, 7: 0}, 20.0, 512),
]


@pytest.mark.parametrize("L,cpl,pins,lam,chi", CASES)
def test_profiles_equal_ed(ctx, L, cpl, pins, lam, chi):
    e = run(ctx, L, lib.BC_OPEN_ZERO_FLUX, cpl, chi, pins, lam)
    e0, (charge, flux) = ed_reference(L, cpl, pins, lam)
    assert abs(e - e0) < 1e-10 * max(1.0, abs(e0)), (e, e0)
    q, f = ctx.site_fluxes()
    assert np.abs(q - charge).max() < 1e-8
    assert np.abs(f - flux).max() < 1e-8
    for axis in range(3):
        qc, ec = ctx.plane_profiles(axis)
        oq, oe = obs.plane_profiles(L, charge, flux, axis)
        assert np.abs(qc - oq).max() < 1e-8, axis
        assert np.abs(ec - oe).max() < 1e-8, axis
    sig = ctx.surface_density()
    assert np.abs(sig - obs.surface_density(L, charge)).max() < 1e-8
    if pins:
        for s, qv in pins.items():
            assert abs(q[s] - qv) < 1e-2, (s, q[s], qv)


@pytest.mark.parametrize("r", [1, 3, 5])
def test_static_potential_equals_ed(ctx, r):
    """V(r) = E(r) - E_0 of two pinned opposite charges along a line, from
    two sweeps, equals the ED difference."""
    L = (8, 1, 1)
    cpl = Couplings(t=0.5, m=1.0, g2e=1.0, g2m=0.0)
    pins = {2: +1, 2 + r: -1}
    e_r = run(ctx, L, lib.BC_OPEN_ZERO_FLUX, cpl, 64, pins, 20.0)
    e_0 = run(ctx, L, lib.BC_OPEN_ZERO_FLUX, cpl, 64)
    o_r, _ = ed_reference(L, cpl, pins, 20.0)
    o_0, _ = ed_reference(L, cpl)
    assert abs((e_r - e_0) - (o_r - o_0)) < 1e-9, (e_r - e_0, o_r - o_0)


def test_free_flux_gauss_relations(ctx):
    """Free flux, Q = 1 on 2x2x1: ground states are degenerate (conserved
    dangling fluxes), so the profiles are checked against Gauss's law with
    the transverse dangling flux of each plane."""
    L = (2, 2, 1)
    run(ctx, L, lib.BC_OPEN_FREE_FLUX, CPL, 64, Q=1)
    q, f = ctx.site_fluxes()
    assert np.abs(f.sum(axis=1) - q).max() < 1e-9
    assert abs(q.sum() - 1.0) < 1e-9
    lat = Lattice(*L)
    for axis in range(3):
        qc, ec = ctx.plane_profiles(axis)
        oq, oe = obs.plane_profiles(L, q, f, axis)
        assert np.abs(qc - oq).max() < 1e-12 and np.abs(ec - oe).max() < 1e-12
        A = lat.nsites // L[axis]
        trans = np.zeros(L[axis])
        for s in range(lat.nsites):
            trans[lat.coords(s)[axis]] += sum(f[s, h] for h in range(6) if h % 3 != axis)
        assert np.abs(np.diff(ec) - qc + 2.0 * trans / A).max() < 1e-9


def link_defects(L, f, axis):
    """Per plane d: sum of (2 - rishon number) over the links that enter
    plane d along `axis` and the links inside it; zero when every link
    obeys the constraint the penalty enforces."""
    lat = Lattice(*L)
    out = np.zeros(L[axis])
    for (x, mu, y) in lat.links():
        dy = lat.coords(y)[axis]
        out[dy] += f[x, 3 + mu] + f[y, mu]
    return out


def test_gauss_relations_4x4x4(ctx):
    """At 4x4x4 (d = 267 in the bulk, no ED): Gauss's law per site; per
    plane it closes with the link defects (2 - L), which the penalty keeps
    small after one sweep; the surface-density sum rule; the shell count."""
    L = (4, 4, 4)
    run(ctx, L, lib.BC_OPEN_ZERO_FLUX, CPL, 16, sweeps=1)
    q, f = ctx.site_fluxes()
    assert np.abs(f.sum(axis=1) - q).max() < 1e-9
    assert abs(q.sum()) < 1e-9
    dL = ctx.observables()["deltaL"]
    for axis in range(3):
        qc, ec = ctx.plane_profiles(axis)
        assert abs(ec[0]) < 1e-12 and abs(ec[-1]) < 1e-12
        A = 16
        res = np.diff(ec) - qc
        assert np.abs(res + 2.0 * link_defects(L, f, axis) / A).max() < 1e-9
        assert np.abs(res).max() <= 2.0 * dL / A + 1e-9
        oq, oe = obs.plane_profiles(L, q, f, axis)
        assert np.abs(qc - oq).max() < 1e-12 and np.abs(ec - oe).max() < 1e-12
    sig = ctx.surface_density()
    assert sig.shape == (2,)
    assert abs(56 * sig[0] + 8 * sig[1] - q.sum()) < 1e-9
    assert np.abs(sig - obs.surface_density(L, q)).max() < 1e-12


def test_periodic_ring_profiles_equal_ed(ctx):
    """A pinned pair on a periodic ring of 8 sites: profiles equal ED's and
    the two face entries (the wrapped link) coincide."""
    L = (8, 1, 1)
    cpl = Couplings(t=0.5, m=1.5, g2e=1.0, g2m=0.0)
    pins = {2: +1, 5: -1}
    e = run(ctx, L, lib.BC_PERIODIC, cpl, 64, pins, 20.0)
    e0, (charge, flux) = ed_reference(L, cpl, pins, 20.0, boundary="periodic")
    assert abs(e - e0) < 1e-10 * max(1.0, abs(e0)), (e, e0)
    q, f = ctx.site_fluxes()
    assert np.abs(q - charge).max() < 1e-8 and np.abs(f - flux).max() < 1e-8
    qc, ec = ctx.plane_profiles(0)
    oq, oe = obs.plane_profiles(L, charge, flux, 0)
    assert np.abs(qc - oq).max() < 1e-8 and np.abs(ec - oe).max() < 1e-8
    assert abs(ec[0] - ec[-1]) < 1e-12
    # the string takes the short way round (3 links, not 5)
    assert np.all(ec[3:6] > 1.5) and np.all(np.abs(ec[[0, 1, 7, 8]]) < 0.2)
    assert np.abs(np.diff(ec) - qc).max() < 1e-9
