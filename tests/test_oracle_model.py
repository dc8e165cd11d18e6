"""Pins of the oracle's model layer (basis, operators, Hamiltonian) against
what the paper and exact diagonalisation fix."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fermions
from oracle.basis import charge_sectors, enumerate_states, site_basis
from oracle.ed import DressedED, OriginalED, dense_dressed_hamiltonian, product_charges
from oracle.hamiltonian import Couplings, Hamiltonian, physical_line
from oracle.lattice import Lattice


# -- dressed-site basis (Methods, local basis and its Gauss law) ---------
def test_bulk_basis_267_from_1458():
    assert 2 * 3 ** 6 == 1458
    for p in (0, 1):
        rows = enumerate_states(p)
        assert rows.shape == (267, 7)
        # Gauss law: phi + sum k = 6 + p on every row, and all entries valid
        assert np.all(rows[:, 0] + rows[:, 1:].sum(1) == 6 + p)
        assert set(np.unique(rows[:, 0])) <= {0, 1}
        assert set(np.unique(rows[:, 1:])) <= {0, 1, 2}
        # canonical order: strictly ascending lexicographic rows
        assert all(tuple(a) < tuple(b) for a, b in zip(rows[:-1], rows[1:]))


def test_bulk_sectors_brute_force():
    # brute force over all 1458 product states, independent of the filter
    for p, expect in ((0, [(0, 141), (1, 126)]), (1, [(-1, 126), (0, 141)])):
        cnt = {}
        for s in range(1458):
            phi, rest = s % 2, s // 2
            ks = [(rest // 3 ** j) % 3 for j in range(6)]
            if phi + sum(ks) == 6 + p:
                cnt[phi - p] = cnt.get(phi - p, 0) + 1
        assert sorted(cnt.items()) == expect
        assert charge_sectors(enumerate_states(p), p) == expect


@pytest.mark.parametrize("f,d", [(0, 1), (1, 2), (2, 5), (3, 13), (4, 35), (5, 96), (6, 267)])
def test_zero_flux_boundary_dims(f, d):
    frozen = tuple(j >= f for j in range(6))
    for p in (0, 1):
        assert len(enumerate_states(p, frozen)) == d


# -- rishon link: the paper's printed action of U and E on link states ---
def test_link_states_and_ladder():
    # modes: a_x=0, b_x=1, a_y=2, b_y=3 (half-link x,+mu then x+mu,-mu)
    nm = 4
    cr = [fermions.creator(m, nm) for m in range(nm)]
    vac = np.zeros(1 << nm); vac[0] = 1.0

    def half(k, a, b, v):
        if k >= 1:
            v = cr[a] @ v
        if k == 2:
            v = cr[b] @ v
        return v

    def ket(kx, ky):
        return half(kx, 0, 1, half(ky, 2, 3, vac))

    right = -ket(0, 2)      # E = +1
    zero = ket(1, 1)        # E = 0
    left = ket(2, 0)        # E = -1
    # the paper writes |right> also as a^dag_y b^dag_y |0>
    assert np.allclose(right, cr[2] @ (cr[3] @ vac))
    eta_x = fermions.rishon_dag(0, 1, nm).T
    etad_y = fermions.rishon_dag(2, 3, nm)
    U = (eta_x @ etad_y).toarray()
    assert np.allclose(U @ left, zero)
    assert np.allclose(U @ zero, right)
    assert np.allclose(U @ right, 0.0)
    nx = (fermions.number(0, nm) + fermions.number(1, nm)).toarray()
    E = np.eye(1 << nm) - nx
    for v, e in ((right, 1), (zero, 0), (left, -1)):
        assert np.allclose(E @ v, e * v)
    L = sum(fermions.number(m, nm) for m in range(nm)).toarray()
    for v in (right, zero, left):
        assert np.allclose(L @ v, 2 * v)
    # eta is 3-hardcore: eta^3 = 0, eta^2 != 0
    ed = fermions.rishon_dag(0, 1, nm).toarray()
    assert np.abs(ed @ ed).max() > 0.5
    assert np.abs(ed @ ed @ ed).max() == 0.0


def test_local_operator_charges():
    rows = enumerate_states(0)
    so = fermions.SiteOps(rows)
    q = rows[:, 0]
    for j in range(6):
        M = so.word([("etad", j), ("psi", None)])
        r, c = np.nonzero(M)
        assert len(r) > 0 and np.all(q[r] - q[c] == -1)
        for i in range(6):
            if i == j:
                continue
            C = so.word([("etad", i), ("eta", j)])
            r, c = np.nonzero(C)
            assert len(r) > 0 and np.all(q[r] == q[c])
            assert set(np.unique(C)) <= {-1.0, 0.0, 1.0}


# -- two formulations of the same model (pins every fermionic sign) ------
CPL = Couplings(t=1.0, m=0.7, g2e=1.3, g2m=0.9)


@pytest.mark.parametrize("L", [(2, 1, 1), (2, 2, 1), (1, 2, 2)])
def test_dressed_equals_original_small(L):
    lat = Lattice(*L)
    o = OriginalED(lat, CPL)
    d = DressedED(Hamiltonian(lat, CPL))
    assert o.dim == d.dim
    assert np.abs(o.spectrum() - d.spectrum()).max() < 1e-12


@pytest.mark.slow
def test_dressed_equals_original_2x2x2():
    lat = Lattice(2, 2, 2)
    o = OriginalED(lat, CPL)
    d = DressedED(Hamiltonian(lat, CPL))
    assert o.dim == d.dim == 3197
    assert np.abs(o.spectrum() - d.spectrum()).max() < 1e-11


def test_free_flux_sectors_match():
    lat = Lattice(2, 2, 1, boundary="free_flux")
    ham = Hamiltonian(lat, CPL)
    dang = [(s, j) for s in range(lat.nsites) for j in range(6) if not lat.present(s)[j]]
    rng = np.random.default_rng(7)
    done = 0
    for _ in range(60):
        fix = {sj: int(rng.choice([-1, 0, 0, 0, 1])) for sj in dang}
        Q = sum(fix.values())
        o = OriginalED(lat, CPL, Q=Q, dangling=fix)
        d = DressedED(ham, Q=Q, dangling=fix)
        assert o.dim == d.dim
        if o.dim:
            assert np.abs(o.spectrum() - d.spectrum()).max() < 1e-12
            done += 1
    assert done >= 5


def test_planted_plaquette_sign_is_caught():
    """Flipping the sign of the plaquette terms (a plausible mistake in the
    four-corner regrouping) must change the spectrum."""
    lat = Lattice(2, 2, 1)
    ham = Hamiltonian(lat, CPL)
    good = DressedED(ham).spectrum()
    ham.terms = [
        (-c if len(ops) == 4 else c, cls, ops) for (c, cls, ops) in ham.terms
    ]
    bad = DressedED(ham).spectrum()
    assert np.abs(good - OriginalED(lat, CPL).spectrum()).max() < 1e-12
    assert np.abs(bad - good).max() > 1e-3


def test_planted_hopping_sign_is_caught():
    lat = Lattice(2, 2, 1)
    ham = Hamiltonian(lat, CPL)
    links = lat.links()
    # flip the hopping on one link only (a wrong Jordan-Wigner sign)
    x, mu, y = links[0]
    flipped = []
    for c, cls, ops in ham.terms:
        sites = tuple(s for s, _ in ops)
        is_hop = len(ops) == 2 and cls == "phys"
        if is_hop and set(sites) == {x, y}:
            c = -c
        flipped.append((c, cls, ops))
    ham.terms = flipped
    bad = DressedED(ham).spectrum()
    assert np.abs(bad - OriginalED(lat, CPL).spectrum()).max() > 1e-3


# -- closed forms --------------------------------------------------------
@pytest.mark.parametrize("m,g2e,t", [(1.0, 2.0, 1.0), (0.7, 1.3, 1.0), (-0.4, 0.5, 0.8)])
def test_two_site_closed_form(m, g2e, t):
    # states {vacuum, pair}: H = [[-m, -t], [-t, m + g_e^2/2]]
    c = Couplings(t=t, m=m, g2e=g2e, g2m=0.0)
    lat = Lattice(2, 1, 1)
    e0 = g2e / 4 - np.sqrt((m + g2e / 4) ** 2 + t ** 2)
    assert abs(DressedED(Hamiltonian(lat, c)).spectrum()[0] - e0) < 1e-13
    assert abs(OriginalED(lat, c).spectrum()[0] - e0) < 1e-13
    # U = S^+/s normalisation gives sqrt(2) t instead: the two readings differ
    e_spin = g2e / 4 - np.sqrt((m + g2e / 4) ** 2 + 2 * t ** 2)
    assert abs(OriginalED(lat, c, ladder="spin").spectrum()[0] - e_spin) < 1e-13
    if m == 1.0:
        assert abs(e0 - (-1.302776)) < 1e-6
        assert abs(e_spin - (-1.561553)) < 1e-6


@pytest.mark.parametrize("g2e,g2m,m", [(1.0, 8.0, 1.0), (2.0, 1.0, -0.3)])
def test_single_plaquette_pure_gauge(g2e, g2m, m):
    c = Couplings(t=0.0, m=m, g2e=g2e, g2m=g2m)
    lat = Lattice(2, 2, 1)
    spec = DressedED(Hamiltonian(lat, c)).spectrum()
    # matter frozen in the bare vacuum only while it is the cheaper sector
    e_loop = g2e - np.sqrt(g2e ** 2 + g2m ** 2 / 2) - 2 * m
    assert np.any(np.abs(spec - e_loop) < 1e-12)


@pytest.mark.parametrize("m", [-2.0, -0.8, -0.3, 0.4, 1.5])
def test_t0_vacuum_vs_charge_crystal(m):
    """t = 0, g_m = 0: E_v = -m N/2, E_ch = (m + g_e^2/2) N/2, level
    crossing at m = -g_e^2/4 (Methods, critical points)."""
    g2e = 2.0
    c = Couplings(t=0.0, m=m, g2e=g2e, g2m=0.0)
    lat = Lattice(2, 2, 1)
    N = lat.nsites
    e0 = DressedED(Hamiltonian(lat, c)).spectrum()[0]
    ev, ech = -m * N / 2, (m + g2e / 2) * N / 2
    assert abs(e0 - min(ev, ech)) < 1e-12
    assert (ev < ech) == (m > -g2e / 4)


def test_physical_line():
    g2e, g2m = physical_line(1.0)
    assert (g2e, g2m) == (1.0, 8.0)
    g2e, g2m = physical_line(2.0, t=1.0)
    assert abs(np.sqrt(g2e * g2m) - 2 * np.sqrt(2)) < 1e-15


# -- penalty exactness ---------------------------------------------------
def test_penalty_recovers_physical_ground_state():
    lat = Lattice(2, 2, 1)
    ham = Hamiltonian(lat, CPL)
    e_phys = OriginalED(lat, CPL).spectrum()[0]
    q = product_charges(ham)
    idx = np.nonzero(q == 0)[0]
    H0 = dense_dressed_hamiltonian(ham, 0.0)[np.ix_(idx, idx)]
    # the product space holds link-violating states besides the 13 physical
    assert len(idx) > 13
    assert np.linalg.eigvalsh(H0)[0] <= e_phys + 1e-12
    H = dense_dressed_hamiltonian(ham, 20.0)[np.ix_(idx, idx)]
    assert np.abs(H - H.T).max() == 0.0
    w = np.linalg.eigvalsh(H)
    assert abs(w[0] - e_phys) < 1e-12
    # the physical spectrum sits below the penalised states, and the
    # penalised states are lifted by at least nu
    phys = OriginalED(lat, CPL).spectrum()
    assert np.abs(w[:13] - phys).max() < 1e-12
    assert w[13] > phys[-1]


def test_hamiltonian_is_symmetric_and_gauss_preserving():
    lat = Lattice(2, 2, 1)
    ham = Hamiltonian(lat, CPL)
    H = dense_dressed_hamiltonian(ham, 3.0)
    assert np.abs(H - H.T).max() < 1e-14
    q = product_charges(ham)
    r, c = np.nonzero(np.abs(H) > 0)
    assert np.all(q[r] == q[c])


# -- local chemical potentials ---------------------------------------------
@pytest.mark.parametrize("mu0,mu1", [(0.3, -0.2), (-1.5, 2.0)])
def test_chemical_potential_two_site_closed_form(mu0, mu1):
    # vacuum phi = (0, 1), pair phi = (1, 0):
    # H = [[-m + mu1, -t], [-t, m + g_e^2/2 + mu0]]
    m, g2e, t = 0.7, 1.3, 0.9
    c = Couplings(t=t, m=m, g2e=g2e, g2m=0.0, mu=(mu0, mu1))
    lat = Lattice(2, 1, 1)
    a, d = -m + mu1, m + 0.5 * g2e + mu0
    e0 = 0.5 * (a + d) - np.sqrt(0.25 * (d - a) ** 2 + t ** 2)
    assert abs(DressedED(Hamiltonian(lat, c)).spectrum()[0] - e0) < 1e-13
    assert abs(OriginalED(lat, c).spectrum()[0] - e0) < 1e-13


def test_chemical_potential_both_formulations_2x2x1():
    mu = tuple(np.random.default_rng(3).uniform(-1.0, 1.0, 4))
    c = Couplings(t=1.0, m=0.7, g2e=1.3, g2m=0.9, mu=mu)
    lat = Lattice(2, 2, 1)
    o, d = OriginalED(lat, c).spectrum(), DressedED(Hamiltonian(lat, c)).spectrum()
    assert np.abs(o - d).max() < 1e-12
    # and the potentials matter
    assert abs(o[0] - OriginalED(lat, CPL).spectrum()[0]) > 1e-3


# -- periodic boundaries -----------------------------------------------------
@pytest.mark.parametrize("L,nlinks,nplaq", [((2, 1, 1), 2, 0), ((4, 1, 1), 4, 0), ((2, 2, 1), 8, 4),
                                            ((2, 2, 2), 24, 24), ((4, 4, 4), 192, 192),
                                            ((4, 2, 1), 16, 8)])
def test_periodic_geometry(L, nlinks, nplaq):
    lat = Lattice(*L, boundary="periodic")
    links = lat.links()
    assert len(links) == nlinks
    assert len(set((x, mu) for x, mu, _ in links)) == nlinks
    assert len(lat.plaquettes()) == nplaq
    for s in range(lat.nsites):
        for a in range(3):
            if L[a] >= 2:
                # the wrap closes every axis
                y = s
                for _ in range(L[a]):
                    y = lat.neighbour(y, 3 + a)
                assert y == s
                assert lat.neighbour(lat.neighbour(s, 3 + a), a) == s
            else:
                assert lat.neighbour(s, a) is None and lat.neighbour(s, 3 + a) is None
    # bulk sites everywhere when every extent is >= 2
    if min(L) >= 2:
        assert all(site_basis(lat, s).shape[0] == 267 for s in range(lat.nsites))


@pytest.mark.parametrize("L", [(2, 1, 1), (4, 1, 1), (2, 2, 1), (1, 2, 2)])
def test_periodic_dressed_equals_original(L):
    """Wrapped hopping and plaquettes (and the doubled links of extent-2
    axes) carry the same signs in both formulations."""
    lat = Lattice(*L, boundary="periodic")
    o = OriginalED(lat, CPL).spectrum()
    d = DressedED(Hamiltonian(lat, CPL)).spectrum()
    assert len(o) == len(d)
    assert np.abs(o - d).max() < 1e-11
    # the wrap matters: the spectrum differs from the open lattice's
    assert abs(o[0] - OriginalED(Lattice(*L), CPL).spectrum()[0]) > 1e-3


def test_periodic_charged_sector_is_empty():
    lat = Lattice(2, 2, 1, boundary="periodic")
    assert OriginalED(lat, CPL, Q=1).dim == 0
    assert DressedED(Hamiltonian(lat, CPL), Q=1).dim == 0


@pytest.mark.parametrize("L", [(4, 1, 1), (2, 2, 1)])
@pytest.mark.parametrize("m", [-2.0, -0.3, 0.4])
def test_periodic_t0_vacuum_vs_charge_crystal(L, m):
    """t = 0, g_m = 0 with periodic boundaries: E_v = -m N/2 and the crystal
    pairs every charge with a neighbour by one unit of flux,
    E_ch = (m + g_e^2/2) N/2."""
    g2e = 2.0
    c = Couplings(t=0.0, m=m, g2e=g2e, g2m=0.0)
    lat = Lattice(*L, boundary="periodic")
    N = lat.nsites
    e0 = DressedED(Hamiltonian(lat, c)).spectrum()[0]
    assert abs(e0 - min(-m * N / 2, (m + g2e / 2) * N / 2)) < 1e-12
