"""Pins of the oracle's tensor layer: block tables, H_eff, Lanczos, the
tree tensor network and its observables."""

import itertools

import numpy as np
import pytest

from oracle import blocks, heff, lanczos
from oracle.ed import DressedED, OriginalED
from oracle.hamiltonian import Couplings, Hamiltonian
from oracle.lattice import Lattice
from oracle.ttn import TTN, Tree, allocate_sectors, default_nu_max, penalty_schedule
from paper_2011_10658_amd import synth

C1 = synth.C1_LEG
C4 = synth.C4_LEG


# -- block tables --------------------------------------------------------
def _brute_table(l, r, p, flux=0):
    out = []
    for (il, (ql, nl)), (ir, (qr, nr)) in itertools.product(enumerate(l), enumerate(r)):
        for ip, (qp, np_) in enumerate(p):
            if ql + qr - qp == flux:
                out.append(((ql, qr), (il, ir, ip), nl * nr * np_))
    out.sort()
    return [t for _, t, _ in out], [s for _, _, s in out]


@pytest.mark.parametrize("legs,nblk,size", [((C1, C1, C1), 19, 792), ((C4, C4, C4), 61, 253604)])
def test_block_table_counts(legs, nblk, size):
    trip, offs = blocks.block_table(*legs)
    assert len(trip) == nblk and offs[-1] == size
    bt, bs = _brute_table(*legs)
    assert trip == bt
    assert list(np.diff(offs)) == bs


def test_block_table_flux_and_roundtrip():
    l = [(-1, 2), (0, 3), (2, 1)]
    r = [(0, 2), (1, 1)]
    p = [(-1, 2), (0, 1), (1, 3), (3, 2)]
    for f in (-1, 0, 1, 2):
        trip, offs = blocks.block_table(l, r, p, f)
        bt, bs = _brute_table(l, r, p, f)
        assert trip == bt
        x = np.arange(offs[-1], dtype=float) + 1.0
        D = blocks.to_dense(x, l, r, p, f)
        assert np.count_nonzero(D) == offs[-1]
        assert np.all(D[~blocks.allowed_mask(l, r, p, f)] == 0)
        assert np.array_equal(blocks.from_dense(D, l, r, p, f), x)
    # in-block index is (i_l * n_r + i_r) * n_p + i_p
    trip, offs = blocks.block_table(l, r, p, 0)
    x = np.arange(offs[-1], dtype=float)
    D = blocks.to_dense(x, l, r, p, 0)
    ol, orr, op = blocks.leg_offsets(l), blocks.leg_offsets(r), blocks.leg_offsets(p)
    for b, (il, ir, ip) in enumerate(trip):
        (ql, nl), (qr, nr), (qp, npp) = l[il], r[ir], p[ip]
        for i, j, k in itertools.product(range(nl), range(nr), range(npp)):
            assert D[ol[ql] + i, orr[qr] + j, op[qp] + k] == offs[b] + (i * nr + j) * npp + k


# -- H_eff ---------------------------------------------------------------
def _dense_terms(terms, leg):
    return [(c, *(blocks.op_to_dense(o, leg, 0) for o in ops)) for c, *ops in terms]


def test_heff_brute_force_tiny():
    leg = [(-1, 2), (0, 2), (1, 1)]
    terms = synth.single_node_terms(5, 2, leg)
    dterms = _dense_terms(terms, leg)
    mask = blocks.allowed_mask(leg, leg, leg)
    rng = np.random.default_rng(0)
    xd = rng.standard_normal(mask.shape) * mask
    y = heff.apply_dense(xd, dterms)
    # index-by-index sum of the definition
    n = mask.shape[0]
    yb = np.zeros_like(xd)
    for c, A, B, C in dterms:
        for i, j, k, a, b, cc in itertools.product(range(n), repeat=6):
            yb[i, j, k] += c * A[i, a] * B[j, b] * C[k, cc] * xd[a, b, cc]
    assert np.abs(y - yb).max() < 1e-12
    assert np.abs(y[~mask]).max() < 1e-15


def test_heff_c1_symmetric_and_flops():
    terms = synth.single_node_terms(1, 8, C1)
    dterms = _dense_terms(terms, C1)
    legs = (C1, C1, C1)
    H = heff.matrix(legs, dterms)
    assert H.shape == (792, 792)
    assert np.array_equal(H, H.T)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(792), rng.standard_normal(792)
    hu, hv = heff.apply_flat(u, legs, dterms), heff.apply_flat(v, legs, dterms)
    assert abs(u @ hv - hu @ v) <= 1e-13 * np.linalg.norm(hu) * np.linalg.norm(v)
    metas = [(True, 0, True, 0, True, 0)] * 8
    assert heff.flops(legs, metas) == 161280
    assert heff.flops(legs, metas[:1]) == 20160


def test_heff_flops_charge_shifted_hand_count():
    """The flop count of charge-shifting terms, counted by hand from the
    mode-product definition (factor on p first, then r, then l, each
    dense on the extents the previous step produced; 2 flops per
    multiply-add; a term whose output block does not exist costs 0).
    Legs l = {0: 2, 1: 3}, r = {0: 1, 1: 2}, p = {0: 2, 1: 4, 2: 1};
    allowed blocks (q_l, q_r, q_p): (0,0,0) (0,1,1) (1,0,1) (1,1,2)."""
    l = [(0, 2), (1, 3)]
    r = [(0, 1), (1, 2)]
    p = [(0, 2), (1, 4), (2, 1)]
    legs = (l, r, p)
    # T1: A shift +1 on l, C shift +1 on p, no factor on r.
    #   (0,0,0) -> (1,0,1): C 2*2*1*2*4 = 32, A 2*2*3*1*4 = 48  -> 80
    #   (0,1,1) -> (1,1,2): C 2*2*2*4*1 = 32, A 2*2*3*2*1 = 24  -> 56
    #   (1,*,*) -> q_l = 2 does not exist                       ->  0
    t1 = (True, 1, False, 0, True, 1)
    assert heff.flops(legs, [t1]) == 136
    # T2: B shift -1 on r, C shift -1 on p.
    #   (0,0,0), (1,0,1) -> q_r = -1 does not exist             ->  0
    #   (0,1,1) -> (0,0,0): C 2*2*2*4*2 = 64, B 2*2*2*1*2 = 16  -> 80
    #   (1,1,2) -> (1,0,1): C 2*3*2*1*4 = 48, B 2*3*2*1*4 = 48  -> 96
    t2 = (False, 0, True, -1, True, -1)
    assert heff.flops(legs, [t2]) == 176
    # T3: A shift +1, B shift -1, C sector preserving.
    #   only (0,1,1) -> (1,0,1): C 2*2*2*4*4 = 128, B 2*2*2*1*4 = 32,
    #   A 2*2*3*1*4 = 48                                         -> 208
    t3 = (True, 1, True, -1, True, 0)
    assert heff.flops(legs, [t3]) == 208
    assert heff.flops(legs, [t1, t2, t3]) == 520
    # the sector-preserving closed form 2 n_l n_r n_p (n_l + n_r + n_p)
    # summed over the four blocks
    t0 = (True, 0, True, 0, True, 0)
    closed = sum(2 * a * b * c * (a + b + c) for a, b, c in ((2, 1, 2), (2, 2, 4), (3, 1, 4), (3, 2, 1)))
    assert heff.flops(legs, [t0]) == closed == 2 * (4 * 5 + 16 * 8 + 12 * 8 + 6 * 6)


def test_heff_shifted_factors_stay_in_blocks():
    # a charge-shifting pair delta_A = +1, delta_C = +1 keeps y on allowed blocks
    leg = [(-1, 2), (0, 3), (1, 2)]
    rng = np.random.default_rng(1)
    A = {q: rng.standard_normal((dict(leg)[q + 1], n)) for q, n in leg if q + 1 in dict(leg)}
    C = {q: rng.standard_normal((dict(leg)[q + 1], n)) for q, n in leg if q + 1 in dict(leg)}
    Ad, Cd = blocks.op_to_dense(A, leg, 1), blocks.op_to_dense(C, leg, 1)
    legs = (leg, leg, leg)
    size = int(blocks.allowed_mask(*legs).sum())
    x = rng.standard_normal(size)
    y = heff.apply_flat(x, legs, [(0.5, Ad, None, Cd)])
    assert y.shape == x.shape and np.abs(y).max() > 0


def _shifted_terms(rng, leg):
    """Non-symmetric factors with charge shifts (dA + dB = dC), identities
    included, so that transposes and index orders all matter."""
    sizes = dict(leg)

    def op(delta):
        blk = {q: rng.standard_normal((sizes[q + delta], n)) for q, n in leg if q + delta in sizes}
        return blocks.op_to_dense(blk, leg, delta), delta

    specs = [((1, 0, 1), 0.7), ((0, 0, 0), -1.3), ((None, -1, -1), 0.4), ((0, None, None), 2.0),
             ((-1, 1, None), 0.9)]
    terms, shifts = [], []
    for sh, c in specs:
        fs = [None if d is None else op(d)[0] for d in sh]
        terms.append((c, *fs))
        shifts.append(sh)
    return terms, shifts


def _adjoint_case(seed=2):
    leg = [(-1, 2), (0, 3), (1, 2)]
    legs = (leg, leg, leg)
    rng = np.random.default_rng(seed)
    terms, shifts = _shifted_terms(rng, leg)
    mask = blocks.allowed_mask(*legs)
    size = int(mask.sum())
    x, yb = rng.standard_normal(size), rng.standard_normal(size)
    return leg, legs, terms, shifts, x, yb


def test_adjoint_x_is_the_transposed_matrix():
    leg, legs, terms, _, x, yb = _adjoint_case()
    H = heff.matrix(legs, terms)
    assert np.abs(H - H.T).max() > 1e-3          # a genuinely non-symmetric case
    xbar, _, _ = heff.adjoint_dense(blocks.to_dense(x, *legs), blocks.to_dense(yb, *legs), terms)
    assert np.abs(blocks.from_dense(xbar, *legs) - H.T @ yb).max() < 1e-12


def test_adjoint_factor_and_coefficient_grads_by_linearity():
    """<ybar, y> is linear in each factor and coefficient, so the change
    along a direction equals the directional derivative exactly."""
    leg, legs, terms, shifts, x, yb = _adjoint_case(5)
    xd, ybd = blocks.to_dense(x, *legs), blocks.to_dense(yb, *legs)
    _, grads, cbar = heff.adjoint_dense(xd, ybd, terms)
    f0 = float(np.sum(ybd * heff.apply_dense(xd, terms)))
    rng = np.random.default_rng(9)
    checked = 0
    for k, (c, *fs) in enumerate(terms):
        for e in range(3):
            if fs[e] is None:
                assert grads[k][e] is None
                continue
            d = shifts[k][e]
            D = blocks.op_to_dense({q: rng.standard_normal(M.shape) for q, M in
                                    blocks.op_from_dense(fs[e], leg, d).items()}, leg, d)
            moved = list(terms)
            nf = list(fs)
            nf[e] = fs[e] + D
            moved[k] = (c, *nf)
            f1 = float(np.sum(ybd * heff.apply_dense(xd, moved)))
            assert abs((f1 - f0) - np.sum(grads[k][e] * D)) < 1e-11 * max(1.0, abs(f1))
            # the gradient lives on the factor's own charge-shift blocks
            G = grads[k][e]
            assert np.abs(G - blocks.op_to_dense(blocks.op_from_dense(G, leg, d), leg, d)).max() == 0
            checked += 1
        moved = list(terms)
        moved[k] = (c + 1.0, *fs)
        f1 = float(np.sum(ybd * heff.apply_dense(xd, moved)))
        assert abs((f1 - f0) - cbar[k]) < 1e-11 * max(1.0, abs(f1))
    assert checked == 11


def test_adjoint_hellmann_feynman_on_lowest_eigenvalue():
    """dE0/dc_k = <v|H_k|v> for the normalised ground state v of a
    symmetric H_eff; the adjoint with x = ybar = v gives it, and central
    differences of the dense eigenvalue agree to O(h^2)."""
    legs = (C1, C1, C1)
    terms = _dense_terms(synth.single_node_terms(4, 3, C1), C1)
    H = heff.matrix(legs, terms)
    w, V = np.linalg.eigh(H)
    v = V[:, 0]
    vd = blocks.to_dense(v, *legs)
    _, _, cbar = heff.adjoint_dense(vd, vd, terms)
    h = 1e-4
    for k in range(3):
        hi = [(c + (h if i == k else 0.0), *f) for i, (c, *f) in enumerate(terms)]
        lo = [(c - (h if i == k else 0.0), *f) for i, (c, *f) in enumerate(terms)]
        fd = (np.linalg.eigvalsh(heff.matrix(legs, hi))[0] -
              np.linalg.eigvalsh(heff.matrix(legs, lo))[0]) / (2 * h)
        assert abs(fd - cbar[k]) < 1e-6


# -- Lanczos -------------------------------------------------------------
def test_lanczos_interlacing_and_convergence():
    terms = synth.single_node_terms(1, 8, C1)
    legs = (C1, C1, C1)
    H = heff.matrix(legs, _dense_terms(terms, C1))
    lam = np.linalg.eigvalsh(H)[0]
    x0 = synth.normal(1, 7, 792)
    prev = np.inf
    for m in (5, 10, 20, 30, 60):
        theta, u, resid, a, b = lanczos.lanczos_cycle(lambda v: H @ v, x0, m)
        assert theta >= lam - 1e-10
        assert theta <= prev + 1e-12
        prev = theta
        # residual estimate equals the true residual of the Ritz pair
        assert abs(np.linalg.norm(H @ u - theta * u) - resid) < 1e-8 * abs(theta)
    theta, u, resid = lanczos.lowest(lambda v: H @ v, x0, m=40, tol=1e-12, max_cycles=20)
    assert abs(theta - lam) < 1e-10 * abs(lam)
    assert u[np.argmax(np.abs(u))] > 0


def test_lanczos_exact_on_small_diagonal():
    d = np.array([3.0, -1.0, 2.0, 0.5])
    theta, u, resid, _, _ = lanczos.lanczos_cycle(lambda v: d * v, np.ones(4), 10)
    assert abs(theta + 1.0) < 1e-14
    assert np.allclose(u, [0, 1, 0, 0], atol=1e-12)


# -- tree geometry and sectors ------------------------------------------
def test_tree_shapes():
    t = Tree(Lattice(4, 4, 4))
    assert len(t.nodes) == 63
    layers = [sum(1 for n in t.nodes if n["layer"] == k) for k in range(6)]
    assert layers == [32, 16, 8, 4, 2, 1]
    assert [t.nodes[k]["axis"] for k in (0, 32, 48, 56, 60, 62)] == [0, 1, 2, 0, 1, 2]
    # bottom node merges two x-neighbours
    n0 = t.nodes[0]
    assert (n0["l"], n0["r"]) == (0, 1)
    t2 = Tree(Lattice(2, 1, 1))
    assert len(t2.nodes) == 1
    with pytest.raises(ValueError):
        Tree(Lattice(3, 2, 2))


def _counts(ham):
    out = []
    for s in range(ham.lat.nsites):
        v, c = np.unique(ham.site_charges(s), return_counts=True)
        out.append({int(a): int(b) for a, b in zip(v, c)})
    return out


def test_sector_allocation_invariants():
    lat = Lattice(4, 4, 4, boundary="free_flux")
    counts = [{0: 141, 1: 126} if lat.parity(s) == 0 else {-1: 126, 0: 141}
              for s in range(lat.nsites)]
    tree = Tree(lat)
    for Q, chi in ((8, 256), (0, 64)):
        legs = allocate_sectors(tree, counts, Q, chi)
        for e, leg in legs.items():
            qs = [q for q, _ in leg]
            assert qs == sorted(set(qs))
            assert all(n > 0 for _, n in leg)
            if e >= lat.nsites and e != tree.top:
                assert sum(n for _, n in leg) <= chi
        assert legs[tree.top] == [(Q, 1)]
        for nd in tree.nodes:
            L, R, P = (dict(legs[nd[k]]) for k in ("l", "r", "p"))
            for q, n in P.items():
                assert n <= sum(L[a] * R.get(q - a, 0) for a in L)
            for q, n in L.items():
                if nd["l"] >= lat.nsites:
                    assert n <= sum(R[b] * P.get(q + b, 0) for b in R)


# -- TTN against ED ------------------------------------------------------
CPL = Couplings(t=1.0, m=0.7, g2e=1.3, g2m=0.9)


def _init(tree, legs, seed=11):
    out = {}
    for n, nd in enumerate(tree.nodes):
        _, offs = blocks.block_table(legs[nd["l"]], legs[nd["r"]], legs[nd["p"]])
        out[n] = synth.sym_uniform(seed, n, int(offs[-1]))
    return out


def _make(lat, cpl, Q, chi, seed=11):
    ham = Hamiltonian(lat, cpl)
    tree = Tree(lat)
    legs = allocate_sectors(tree, _counts(ham), Q, chi)
    return TTN(ham, Q, chi, init=_init(tree, legs, seed), legs=legs)


@pytest.mark.parametrize("L", [(2, 1, 1), (2, 2, 1)])
def test_ttn_exact_bond_dim_equals_ed(L):
    lat = Lattice(*L)
    e0 = OriginalED(lat, CPL).spectrum()[0]
    T = _make(lat, CPL, 0, 64)
    for _ in range(3):
        E = T.sweep(20.0, m=40, cycles=3, tol=1e-13)
    assert abs(E - e0) < 1e-10 * abs(e0)
    ob = T.observables()
    assert abs(ob["Q"]) < 1e-12
    assert ob["deltaL"] < 1e-9
    # the renormalised energy equals <psi|H|psi> from the full state vector
    psi = _full_state(T)
    ham = T.ham
    from oracle.ed import dense_dressed_hamiltonian
    Hd = dense_dressed_hamiltonian(ham, 20.0)
    assert abs(psi @ Hd @ psi / (psi @ psi) - E) < 1e-10 * abs(E)


def _full_state(T):
    """Contract the whole tree into a product-space vector (site 0 is the
    slowest index, as in the Kronecker order)."""
    tree = T.tree
    vec = {s: (np.eye(T.ham.dims[s]), [s]) for s in range(tree.N)}
    for n, nd in enumerate(tree.nodes):
        Ml, sl = vec[nd["l"]]
        Mr, sr = vec[nd["r"]]
        x = T.nodes[n]
        # M[(sites...), leg]
        M = np.einsum("ua,vb,abc->uvc", Ml, Mr, x).reshape(-1, x.shape[2])
        vec[nd["p"]] = (M, sl + sr)
    M, sites = vec[tree.top]
    dims = [T.ham.dims[s] for s in sites]
    psi = M[:, 0].reshape(dims)
    order = np.argsort(sites)
    return np.transpose(psi, order).reshape(-1)


def test_ttn_isometries_after_sweep():
    T = _make(Lattice(2, 2, 1), CPL, 0, 8)
    T.sweep(5.0, m=20, cycles=1)
    T.move_to(T.tree.root)
    for n in range(len(T.tree.nodes)):
        if n == T.tree.root:
            continue
        x = T.nodes[n]
        G = np.einsum("abc,abd->cd", x, x)
        assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


def test_ttn_variational_bound_2x2x2():
    lat = Lattice(2, 2, 2)
    e0 = OriginalED(lat, CPL).spectrum()[0]
    T = _make(lat, CPL, 0, 16)
    numax = default_nu_max(CPL)
    prev = None
    for s in range(6):
        E = T.sweep(penalty_schedule(s, numax), m=20, cycles=1)
    assert E >= e0 - 1e-9
    ob = T.observables()
    assert abs(ob["Q"]) < 1e-12
    # Gauss law is exact by construction of every basis row
    for s in range(lat.nsites):
        rows = T.ham.rows[s]
        assert np.all(rows[:, 0] + rows[:, 1:].sum(1) == 6 + lat.parity(s))


def test_ttn_t0_closed_form():
    g2e = 2.0
    for m in (-1.5, 1.0):
        c = Couplings(t=0.0, m=m, g2e=g2e, g2m=0.0)
        lat = Lattice(2, 2, 1)
        T = _make(lat, c, 0, 32)
        for s in range(3):
            E = T.sweep(10.0, m=30, cycles=2, tol=1e-13)
        N = lat.nsites
        exact = min(-m * N / 2, (m + g2e / 2) * N / 2)
        assert abs(E - exact) < 1e-9
        ob = T.observables()
        # vacuum at large positive m, full charge crystal at large negative m
        assert abs(ob["rho"] - (0.0 if m > 0 else 1.0)) < 1e-8


def test_ttn_free_flux_nonzero_charge():
    """Finite charge under free-flux boundaries: <Q> is exactly the sector
    charge and the energy is bounded by dressed-site ED with L = 2."""
    lat = Lattice(2, 1, 1, boundary="free_flux")
    T = _make(lat, CPL, 1, 400)
    for _ in range(2):
        E = T.sweep(20.0, m=60, cycles=4, tol=1e-13)
    ob = T.observables()
    assert abs(ob["Q"] - 1.0) < 1e-12
    d = DressedED(T.ham, Q=1)
    e0 = np.linalg.eigvalsh(d.H.toarray())[0]
    assert abs(E - e0) < 1e-9 * max(1.0, abs(e0))


def test_penalty_schedule_shape():
    nus = [penalty_schedule(s, 40.0) for s in range(12)]
    assert abs(nus[0] - 2.0) < 1e-15 and abs(nus[3] - 10.0) < 1e-15
    assert all(b > a for a, b in zip(nus[:8], nus[1:8]))
    assert nus[7] == 40.0 and nus[11] == 40.0
    d = np.diff(nus[3:8])
    assert all(b > a for a, b in zip(d[:-1], d[1:]))  # quadratic stage accelerates


@pytest.mark.parametrize("L", [(2, 1, 1), (4, 1, 1), (8, 1, 1)])
def test_ttn_periodic_exact_bond_dim_equals_ed(L):
    """Periodic boundaries: wrapped links are terms between distant leaves;
    at exact bond dimension the sweep reaches the ED ground state."""
    lat = Lattice(*L, boundary="periodic")
    e0 = OriginalED(lat, CPL).spectrum()[0]
    T = _make(lat, CPL, 0, 64)
    for _ in range(3):
        E = T.sweep(20.0, m=40, cycles=3, tol=1e-13)
    assert abs(E - e0) < 1e-10 * abs(e0)
    assert T.observables()["deltaL"] < 1e-9


# -- subspace expansion ------------------------------------------------------
def _expansion_ttn(L, chi, bc="zero_flux", Q=0, cpl=CPL):
    lat = Lattice(*L, boundary=bc)
    return lat, _make(lat, cpl, Q, chi)


def test_expansion_move_keeps_state_and_isometry():
    """An expansion move enlarges the link with directions that b does not
    see yet: the contracted state is unchanged, a is an isometry toward the
    link, and the link has grown."""
    lat, T = _expansion_ttn((2, 2, 1), 2)
    T.sweep(20.0, m=30, cycles=2, tol=1e-12)
    T.move_to(0)
    T.set_expansion(0.1, 4, 1000, 5)
    T.last_updated = 0                   # as right after an update of node 0
    link = T.tree.nodes[0]["p"]
    before = _full_state(T)
    dim0 = sum(n for _, n in T.legs[link])
    T.move_to(T.tree.root)
    after = _full_state(T)
    assert np.abs(after - before).max() < 1e-12 * np.abs(before).max()
    assert sum(n for _, n in T.legs[link]) > dim0
    # node 0 is an isometry toward its parent leg
    x = T.nodes[0]
    G = np.tensordot(x, x, axes=([0, 1], [0, 1]))
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12


@pytest.mark.parametrize("L,pins", [((2, 2, 1), None), ((4, 1, 1), None),
                                    ((8, 1, 1), {2: 1, 5: -1})])
def test_expansion_reaches_ed_from_small_bond_dimension(L, pins):
    """Bond dimension 2 from the allocation rule cannot hold the ground
    state; with expansion the sweeps grow the links (and their sectors) to
    the ED energy, and the links end at the rank of the state."""
    cpl = CPL
    if pins:
        from oracle.observables import pinning_potentials
        mu = tuple(pinning_potentials(L, pins, 20.0))
        cpl = Couplings(t=0.5, m=1.0, g2e=1.0, g2m=0.0, mu=mu)
    lat = Lattice(*L)
    e0 = OriginalED(lat, cpl).spectrum()[0]
    plain = _make(lat, cpl, 0, 2)
    grown = _make(lat, cpl, 0, 2)
    start = {e: {q for q, _ in leg} for e, leg in grown.legs.items()}
    grown.set_expansion(1e-2, 8, 64, 99)
    for _ in range(8):
        ep = plain.sweep(20.0, m=40, cycles=3, tol=1e-12)
        eg = grown.sweep(20.0, m=40, cycles=3, tol=1e-12)
    assert ep > e0 + 1e-3
    assert abs(eg - e0) < 1e-9 * abs(e0)
    assert grown.observables()["deltaL"] < 1e-9
    if pins:
        # the symmetry sectors adapted: some link carries a charge that the
        # initial allocation did not give it
        assert any({q for q, _ in grown.legs[e]} - start[e] for e in start)


def test_expansion_respects_chi_max_and_bound():
    lat, T = _expansion_ttn((2, 2, 1), 2)
    T.set_expansion(1e-2, 8, 3, 99)
    e0 = OriginalED(lat, CPL).spectrum()[0]
    for _ in range(4):
        E = T.sweep(20.0, m=40, cycles=3, tol=1e-12)
        for e, leg in T.legs.items():
            if e >= lat.nsites:
                assert sum(n for _, n in leg) <= 3
    assert E >= e0 - 1e-10


def test_adaptive_penalty_schedule_hand_values():
    """The adaptive switch of the driven penalty (Methods, "Numerical
    Convergence"), by hand: nu_max = 40, 4 linear + 4 quadratic sweeps, so
    the linear phase runs 2, 14/3, 22/3, 10 (slope 8/3).  Sweep 2's energy
    rises above sweep 1's: the quadratic phase starts at sweep 3 from 22/3
    and reaches 40 in four sweeps: 22/3 + (40 - 22/3) u^2, u = 1/4 .. 1."""
    from oracle.ttn import adaptive_penalty_schedule
    E = [-10.0, -12.0, -11.5, -11.0, -10.0, -9.0, -8.0, -7.0]
    nu = [adaptive_penalty_schedule(s, E[:s], 40.0, 4, 4) for s in range(9)]
    start = 22.0 / 3.0
    want = [2.0, 2.0 + 8.0 / 3.0, start] + [start + (40.0 - start) * (k / 4.0) ** 2 for k in (1, 2, 3, 4)] \
        + [40.0, 40.0]
    assert np.allclose(nu, want, rtol=0, atol=1e-12), (nu, want)
    assert abs(nu[3] - 9.375) < 1e-12 and abs(nu[4] - 15.5) < 1e-12
    # no rise (or one below 1e-10 |E|): the fixed schedule
    E2 = [-10.0, -12.0, -12.0 + 1e-12, -13.0, -14.0, -15.0, -16.0, -17.0]
    for s in range(10):
        assert adaptive_penalty_schedule(s, E2[:s], 40.0, 4, 4) == penalty_schedule(s, 40.0, 4, 4)
    # a rise at the first comparison: quadratic from sweep 2, from nu(1)
    E3 = [-10.0, -9.0]
    assert adaptive_penalty_schedule(1, E3[:1], 40.0, 4, 4) == 2.0 + 8.0 / 3.0
    s1 = 2.0 + 8.0 / 3.0
    assert abs(adaptive_penalty_schedule(2, E3, 40.0, 4, 4) - (s1 + (40.0 - s1) / 16.0)) < 1e-12
