"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol the header declares, and its integer work (local bases, tree
sectors, block tables) is bit-exact against the oracle."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import blocks as oblocks
from oracle.basis import site_basis
from oracle.lattice import Lattice
from oracle.ttn import Tree, allocate_sectors
from paper_2011_10658_amd import lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "qedttn.h")).read()
    names = set(re.findall(r"\b(qed_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 30
    L = lib.load()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(lib.SIGNATURES) <= names


def _oracle_legs(L, bc, Q, chi):
    lat = Lattice(*L, boundary=bc)
    counts, dims = [], []
    for s in range(lat.nsites):
        rows = site_basis(lat, s)
        dims.append(len(rows))
        v, c = np.unique(rows[:, 0] - lat.parity(s), return_counts=True)
        counts.append({int(a): int(b) for a, b in zip(v, c)})
    tree = Tree(lat)
    return tree, dims, allocate_sectors(tree, counts, Q, chi)


@pytest.mark.parametrize(
    "L,bc,Q,chi",
    [((2, 1, 1), 0, 0, 8), ((2, 2, 1), 0, 0, 64), ((2, 2, 2), 0, 0, 16), ((2, 2, 2), 0, 0, 64),
     ((2, 2, 2), 1, 0, 64), ((2, 2, 2), 1, 3, 100), ((4, 4, 4), 1, 8, 256), ((4, 4, 4), 0, 0, 32),
     ((4, 2, 2), 1, -2, 48)])
def test_tree_sectors_bit_exact(L, bc, Q, chi):
    tree, dims, legs = _oracle_legs(L, "zero_flux" if bc == 0 else "free_flux", Q, chi)
    ctx = lib.Context(-1)
    ctx.set_lattice(*L, bc)
    ctx.set_couplings(1.0, 1.0, 1.0, 1.0)
    ctx.set_charge_sector(Q)
    ctx.set_bond_dim(chi)
    ctx.build_hamiltonian()
    nn, ns = ctx.tree()
    assert (nn, ns) == (len(tree.nodes), tree.N)
    assert ctx.local_dims() == dims
    for n, nd in enumerate(tree.nodes):
        assert ctx.node_links(n) == (nd["l"], nd["r"], nd["p"])
    for e in range(tree.nlinks):
        assert ctx.leg_sectors(e) == legs[e], e


def test_bulk_local_dimension():
    ctx = lib.Context(-1)
    ctx.set_lattice(4, 4, 4, lib.BC_OPEN_FREE_FLUX)
    ctx.set_couplings(1.0, 1.0, 1.0, 8.0)
    ctx.build_hamiltonian()
    assert set(ctx.local_dims()) == {267}
    assert ctx.leg_sectors(0) == [(0, 141), (1, 126)]
    assert ctx.leg_sectors(1) == [(-1, 126), (0, 141)]


def test_node_blocks_bit_exact():
    rng = np.random.default_rng(5)
    for trial in range(40):
        legs = []
        for _ in range(3):
            S = int(rng.integers(1, 7))
            qs = sorted(rng.choice(np.arange(-6, 7), S, replace=False).tolist())
            legs.append([(q, int(rng.integers(1, 9))) for q in qs])
        flux = int(rng.integers(-2, 3))
        ot, oo = oblocks.block_table(*legs, flux)
        if not ot:
            continue
        lt, lo = lib.node_blocks(*legs, flux)
        assert lt == ot
        assert np.array_equal(lo, oo)
    t, o = lib.node_blocks(synth.C1_LEG, synth.C1_LEG, synth.C1_LEG)
    assert len(t) == 19 and o[-1] == 792
    t, o = lib.node_blocks(synth.C4_LEG, synth.C4_LEG, synth.C4_LEG)
    assert len(t) == 61 and o[-1] == 253604


def test_error_paths():
    ctx = lib.Context(-1)
    with pytest.raises(lib.QedError) as e:
        ctx.set_lattice(3, 2, 2)
    assert e.value.code == -1
    with pytest.raises(lib.QedError) as e:
        ctx.set_lattice(2, 2, 2, 7)
    assert e.value.code == -1
    with pytest.raises(lib.QedError) as e:
        ctx.build_hamiltonian()
    assert e.value.code == -2
    ctx.set_lattice(2, 2, 2)
    ctx.set_couplings(1, 1, 1, 1)
    ctx.set_charge_sector(1)
    with pytest.raises(lib.QedError) as e:
        ctx.build_hamiltonian()
    assert e.value.code == -1 and "zero-flux" in str(e.value)
    ctx.set_charge_sector(0)
    ctx.build_hamiltonian()
    with pytest.raises(lib.QedError) as e:
        ctx.init_state(1)
    assert e.value.code == -2
    with pytest.raises(lib.QedError):
        ctx.set_lanczos(0)
    with pytest.raises(lib.QedError):
        ctx.set_lanczos_schedule(1e-4, 1.5)
    ctx.set_lanczos_schedule(1e-4, 0.1)
    ctx.set_lanczos_schedule(0.0)
    with pytest.raises(lib.QedError) as e:
        lib.node_blocks([(0, 1), (0, 2)], [(0, 1)], [(0, 1)])
    assert lib.physical_line(1.0) == (1.0, 8.0)
    with pytest.raises(lib.QedError):
        lib.physical_line(0.0)


# -- checkpoint files ---------------------------------------------------------
def _fnv(data):
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _checkpoint_bytes(ctx, L, bc, Q, chi, cpl, nodes_fill=0.25):
    """A well-formed state file for the context's tree, written from the
    documented layout (independent of the library's writer)."""
    import struct
    nn, _ = ctx.tree()
    links = []
    e = 0
    while True:
        try:
            links.append(ctx.leg_sectors(e))
        except lib.QedError:
            break
        e += 1
    body = b"QEDTTNS\x00" + struct.pack("<I", 1)
    body += struct.pack("<6i", *L, bc, Q, chi) + struct.pack("<4d", *cpl)
    body += struct.pack("<iiid", 3, 1, 1, -1.5)
    body += struct.pack("<i", len(links))
    for leg in links:
        body += struct.pack("<i", len(leg))
        for q, n in leg:
            body += struct.pack("<ii", q, n)
    body += struct.pack("<i", nn)
    for n in range(nn):
        l, r, p = [links[k] for k in ctx.node_links(n)]
        size = int(oblocks.block_table(l, r, p)[1][-1])
        body += struct.pack("<q", size) + np.full(size, nodes_fill).tobytes()
    return body + struct.pack("<Q", _fnv(body))


def test_checkpoint_file_checks(tmp_path):
    ctx = lib.Context(-1)
    with pytest.raises(lib.QedError) as e:
        ctx.load_state(str(tmp_path / "missing.ckpt"))
    assert e.value.code == -8
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint at all")
    with pytest.raises(lib.QedError) as e:
        ctx.load_state(str(junk))
    assert e.value.code == -8
    ctx.set_lattice(2, 2, 1, lib.BC_OPEN_ZERO_FLUX)
    ctx.set_couplings(1.0, 1.0, 1.0, 8.0)
    ctx.set_bond_dim(8)
    ctx.build_hamiltonian()
    good = _checkpoint_bytes(ctx, (2, 2, 1), lib.BC_OPEN_ZERO_FLUX, 0, 8, (1.0, 1.0, 1.0, 8.0))
    f = tmp_path / "state.ckpt"
    f.write_bytes(good)
    # a whole file passes every format check and stops only at the device
    with pytest.raises(lib.QedError) as e:
        ctx.load_state(str(f))
    assert e.value.code == -2 and "host-only" in str(e.value)
    # any flipped byte, or a cut, is caught by the checksum or the reader
    for pos in (20, len(good) // 2, len(good) - 3):
        bad = bytearray(good)
        bad[pos] ^= 0x10
        f.write_bytes(bytes(bad))
        with pytest.raises(lib.QedError) as e:
            ctx.load_state(str(f))
        assert e.value.code == -8, pos
    f.write_bytes(good[:-100])
    with pytest.raises(lib.QedError) as e:
        ctx.load_state(str(f))
    assert e.value.code == -8
    with pytest.raises(lib.QedError) as e:
        ctx.save_state(str(tmp_path / "x.ckpt"))
    assert e.value.code == -2


def test_chemical_potential_arguments():
    ctx = lib.Context(-1)
    with pytest.raises(lib.QedError) as e:
        ctx._c(ctx.lib.qed_set_chemical_potential(ctx.h, None))
    assert e.value.code == -2
    ctx.set_lattice(2, 2, 1)
    with pytest.raises(ValueError):
        ctx.set_chemical_potential([0.1, 0.2])
    with pytest.raises(lib.QedError) as e:
        ctx.set_chemical_potential([0.0, float("nan"), 0.0, 0.0])
    assert e.value.code == -1
    ctx.set_chemical_potential([0.1, -0.2, 0.3, 0.0])
    ctx.set_chemical_potential(None)


def test_pin_charges_arguments():
    ctx = lib.Context(-1)
    with pytest.raises(lib.QedError) as e:
        ctx.pin_charges({0: 1}, 10.0)
    assert e.value.code == -2
    ctx.set_lattice(4, 1, 1)
    bad = [({1: +1}, 10.0),          # +1 on an odd site
           ({0: -1}, 10.0),          # -1 on an even site
           ({4: 0}, 10.0),           # site out of range
           ({-1: 0}, 10.0),
           ({0: 2}, 10.0),
           ({0: 1}, 0.0),            # lambda must be positive
           ({0: 1}, float("inf"))]
    for pins, lam in bad:
        with pytest.raises(lib.QedError) as e:
            ctx.pin_charges(pins, lam)
        assert e.value.code == -1, (pins, lam)
    sites = (C.c_int * 2)(0, 0)
    qs = (C.c_int * 2)(1, 1)
    with pytest.raises(lib.QedError) as e:
        ctx._c(ctx.lib.qed_pin_charges(ctx.h, 2, sites, qs, 5.0))
    assert e.value.code == -1
    ctx.pin_charges({0: 1, 1: -1, 2: 0, 3: 0}, 5.0)
    ctx.close()


def test_profile_arguments():
    ctx = lib.Context(-1)
    ctx.set_lattice(2, 2, 1)
    for axis in (-1, 3):
        with pytest.raises(lib.QedError) as e:
            ctx._c(ctx.lib.qed_get_plane_profiles(ctx.h, axis, None, None))
        assert e.value.code == -1
    with pytest.raises(ValueError):
        ctx.plane_profiles(3)
    ctx.close()


@pytest.mark.parametrize("L", [(2, 2, 2), (4, 2, 1), (2, 1, 1), (4, 4, 4)])
def test_periodic_local_dims_and_charge(L):
    """Periodic lattices: local dimensions equal the oracle's bases (267
    wherever every extent is >= 2), and only Q = 0 builds."""
    ctx = lib.Context(-1)
    ctx.set_lattice(*L, lib.BC_PERIODIC)
    ctx.set_couplings(1, 1, 1, 1)
    ctx.set_bond_dim(16)
    ctx.build_hamiltonian()
    lat = Lattice(*L, boundary="periodic")
    want = [site_basis(lat, s).shape[0] for s in range(lat.nsites)]
    assert list(ctx.local_dims()) == want
    ctx.set_charge_sector(2)
    with pytest.raises(lib.QedError) as e:
        ctx.build_hamiltonian()
    assert e.value.code == -1 and "periodic" in str(e.value)
    ctx.close()
