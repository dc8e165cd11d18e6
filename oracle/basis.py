"""Gauge-invariant dressed-site basis (Methods, "Fermionic compact
representation of local gauge-invariant site").

A dressed site holds the staggered matter mode (occupation phi in {0,1})
and six rishon half-links (k_j in {0,1,2}, order -x,-y,-z,+x,+y,+z).
Gauss's law in rishon language (final Gauss-law equation of that section)
fixes   phi + sum_j k_j = 6 + p   with p = (1 - (-1)^x)/2 the site parity.
Without the constraint there are 2 * 3^6 = 1458 states; with it 267.

Canonical order: lexicographic ascending in (phi, k_1, ..., k_6), so the
two U(1) charge sectors (phi = 0 and phi = 1) are contiguous.
Site charge (Results, the Q operator): q = phi - p.

Under the zero-flux boundary reading a half-link with no partner is frozen
at k = 1 (E = 1 - k = 0), which shrinks the basis; under free-flux it stays
a free 3-state mode.  Periodic lattices freeze only the half-links of axes
of extent 1 (every other half-link has a partner).
"""

from itertools import product

import numpy as np


def enumerate_states(parity, frozen=(False,) * 6):
    """All (phi, k1..k6) obeying the local Gauss law, canonical order.

    frozen[j] = True pins k_j = 1 (zero-flux boundary half-link).
    Brute force over the 2*3^6 product states, filtered.
    """
    rows = []
    for phi in (0, 1):
        for ks in product((0, 1, 2), repeat=6):
            if any(frozen[j] and ks[j] != 1 for j in range(6)):
                continue
            if phi + sum(ks) == 6 + parity:
                rows.append((phi,) + ks)
    rows.sort()
    return np.array(rows, dtype=np.int64).reshape(-1, 7)


def site_basis(lat, s):
    """Basis rows for site s of Lattice `lat` (respecting the boundary)."""
    p = lat.parity(s)
    if lat.boundary in ("zero_flux", "periodic"):
        frozen = tuple(not x for x in lat.present(s))
    else:
        frozen = (False,) * 6
    return enumerate_states(p, frozen)


def site_charges(rows, parity):
    """U(1) charge q = phi - p of every basis row."""
    return rows[:, 0] - parity


def charge_sectors(rows, parity):
    """[(q, count)] ascending in q."""
    q = site_charges(rows, parity)
    vals, counts = np.unique(q, return_counts=True)
    return [(int(a), int(b)) for a, b in zip(vals, counts)]
