"""Lattice geometry for the cubic LGT of Eq. 1 (Results, "The model").

Sites x = (i, j, k), 0 <= i < Lx etc.; flat index s = i + Lx*(j + Ly*k).
Site parity p = (i + j + k) mod 2; (-1)^x = 1 - 2p.

Half-links of a site are numbered in the order in which the local
gauge-invariant basis lists them (Methods, local basis equation):
    0: -x   1: -y   2: -z   3: +x   4: +y   5: +z
A link (x, mu) joins the +mu half-link of x with the -mu half-link of x+mu.

Boundary readings (the paper runs open boundaries without stating what
happens to the boundary half-links, see Results "Finite Density"):
    "zero_flux": a half-link pointing out of the lattice is frozen at
                 k = 1 (E = 0); only total charge Q = 0 exists.
    "free_flux": a half-link pointing out of the lattice is a free
                 3-state mode (dangling flux) with electric energy
                 (g_e^2/2) E^2 and no penalty partner.
    "periodic":  every axis of extent >= 2 wraps around (the zero-charge
                 transition runs with periodic boundaries, Results); an
                 axis of extent 1 has no links and its half-links are
                 frozen as under zero flux.  With extent 2 the two sites
                 of an axis are joined by two distinct links (the direct
                 one and the wrapped one).  Only Q = 0 exists.
"""

from itertools import product

AXES = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
BOUNDARY_MODES = ("zero_flux", "free_flux", "periodic")


class Lattice:
    def __init__(self, Lx, Ly, Lz, boundary="zero_flux"):
        if boundary not in BOUNDARY_MODES:
            raise ValueError(boundary)
        self.L = (int(Lx), int(Ly), int(Lz))
        self.boundary = boundary
        self.nsites = Lx * Ly * Lz

    # -- sites ---------------------------------------------------------
    def coords(self, s):
        Lx, Ly, _ = self.L
        return (s % Lx, (s // Lx) % Ly, s // (Lx * Ly))

    def index(self, c):
        Lx, Ly, _ = self.L
        return c[0] + Lx * (c[1] + Ly * c[2])

    def inside(self, c):
        return all(0 <= c[a] < self.L[a] for a in range(3))

    def parity(self, s):
        return sum(self.coords(s)) % 2

    def neighbour(self, s, half):
        """Site across half-link `half` (0..5) or None at the boundary."""
        c = list(self.coords(s))
        a = half % 3
        c[a] += 1 if half >= 3 else -1
        if self.boundary == "periodic" and self.L[a] >= 2:
            c[a] %= self.L[a]
        return self.index(c) if self.inside(c) else None

    # -- links ---------------------------------------------------------
    def links(self):
        """All links as (x, mu, y) with y = x + mu, mu in 0..2."""
        out = []
        for s in range(self.nsites):
            for mu in range(3):
                y = self.neighbour(s, 3 + mu)
                if y is not None:
                    out.append((s, mu, y))
        return out

    def present(self, s):
        """Tuple of 6 bools: is half-link j attached to a link?"""
        return tuple(self.neighbour(s, j) is not None for j in range(6))

    def plaquettes(self):
        """All plaquettes as (x, alpha, beta) with alpha < beta."""
        out = []
        for s in range(self.nsites):
            for al, be in ((0, 1), (0, 2), (1, 2)):
                xa = self.neighbour(s, 3 + al)
                xb = self.neighbour(s, 3 + be)
                if xa is None or xb is None or self.neighbour(xa, 3 + be) is None:
                    continue
                out.append((s, al, be))
        return out

    def all_sites(self):
        return list(range(self.nsites))

    def iter_coords(self):
        Lx, Ly, Lz = self.L
        for k, j, i in product(range(Lz), range(Ly), range(Lx)):
            yield (i, j, k)
