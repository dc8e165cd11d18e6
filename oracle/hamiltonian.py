"""Lattice QED Hamiltonian on dressed sites as a list of site-local terms.

Eq. 1 (Results, "The model"):
    H = -t  sum_{x,mu} (psi_x^dag U_{x,mu} psi_{x+mu} + h.c.)
        + m sum_x (-1)^x psi_x^dag psi_x  [+ sum_x mu_x psi_x^dag psi_x]
        + (g_e^2/2) sum_{x,mu} E_{x,mu}^2
        - (g_m^2/2) sum_x (box_xy + box_xz + box_yz + h.c.)
    box_{a,b} = U_{x,a} U_{x+a,b} U^dag_{x+b,a} U^dag_{x,b}
plus the link penalty (Methods, "Numerical Convergence", penalty eq.)
    H_pen = nu sum_{x,mu} (1 - delta_{2, L_{x,mu}}),
    L_{x,mu} = k_{x,+mu} + k_{x+mu,-mu}  (total rishon number on the link).

Rishon form (Methods): U_{x,mu} = eta_{x,+mu} eta^dag_{x+mu,-mu};
E_{x,mu} = 1 - k_{x,+mu} on the lower site's half-link (exact for L = 2).
Multi-site words are regrouped site by site; the sign of the regrouping is
counted from the number of transpositions of odd operators, so hopping and
plaquette terms come out as products of site-local bosonic matrices
(for the plaquette this reproduces the overall minus sign of the
four-corner product written in the paper).

Readings taken where the paper is silent:
  * E^2 of a link is read on the lower site's +mu half-link.
  * Under the free-flux boundary each dangling half-link j carries
    (g_e^2/2) (1 - k_j)^2 and no penalty.
  * Periodic boundaries: wrapped links get the same hopping, plaquette,
    electric and penalty terms as interior links (the site operators are
    bosonic, so no Jordan-Wigner string crosses the lattice); the
    original-formulation ED, with its explicit fermion signs, pins this.
  * U has unit ladder elements (link-state action in the Methods); the
    alternative S^+/s normalisation is available in the ED module only.
  * The hopping carries no extra staggered phase (none appears in Eq. 1).

Every term is (coef, cls, ((site, matrix), ...)) with sites ascending and
cls in {"phys", "pen"}; the full operator is phys + nu * pen + offsets.
"""

from dataclasses import dataclass

import numpy as np

from .basis import site_basis
from .fermions import SiteOps


@dataclass
class Couplings:
    t: float = 1.0
    m: float = 1.0
    g2e: float = 1.0
    g2m: float = 1.0
    # local chemical potentials mu_x (one per site, or empty for none): the
    # term sum_x mu_x psi_x^dag psi_x that pins charges (Results, the
    # capacitor and confinement set-ups)
    mu: tuple = ()


def physical_line(g2, t=1.0):
    """g_e^2 = g^2 / a, g_m^2 = 8 / (g^2 a) with a = 1/t (Results)."""
    return g2 * t, 8.0 * t / g2


def regroup(word):
    """Split an ordered product of odd single-mode operators into
    per-site words.  word: [(site, kind, j)].  Returns (sign, {site: [...]})
    with each site's operators in their original relative order."""
    sites = sorted({w[0] for w in word})
    order = sorted(range(len(word)), key=lambda i: (sites.index(word[i][0]), i))
    inv = 0
    for a in range(len(order)):
        for b in range(a + 1, len(order)):
            if order[a] > order[b]:
                inv += 1
    groups = {}
    for i in order:
        s, kind, j = word[i]
        groups.setdefault(s, []).append((kind, j))
    return (-1.0) ** inv, groups


def _dagger_word(word):
    flip = {"psi": "psid", "psid": "psi", "eta": "etad", "etad": "eta"}
    return [(s, flip[k], j) for (s, k, j) in reversed(word)]


def _U(x, mu, y):
    """word of U_{x,mu}, y = x + mu"""
    return [(x, "eta", 3 + mu), (y, "etad", mu)]


def _Udag(x, mu, y):
    return _dagger_word(_U(x, mu, y))


class Hamiltonian:
    def __init__(self, lat, cpl):
        self.lat = lat
        self.cpl = cpl
        self.rows = [site_basis(lat, s) for s in range(lat.nsites)]
        self.site_ops = [SiteOps(r) for r in self.rows]
        self.dims = [r.shape[0] for r in self.rows]
        self.terms = []
        self.offset = {"phys": 0.0, "pen": 0.0}
        self._build()

    def _word_term(self, coef, word):
        sign, groups = regroup(word)
        ops = tuple(
            (s, self.site_ops[s].word(groups[s])) for s in sorted(groups)
        )
        self.terms.append((coef * sign, "phys", ops))

    def _build(self):
        lat, c = self.lat, self.cpl
        # onsite: staggered mass + electric energy of links owned by the
        # site's +mu half-links (+ dangling half-links for free flux)
        for s in range(lat.nsites):
            so = self.site_ops[s]
            p = lat.parity(s)
            h = c.m * (1 - 2 * p) * so.phi()
            if c.mu:
                h = h + c.mu[s] * so.phi()
            pres = lat.present(s)
            for j in range(6):
                Ej = np.eye(so.d) - so.kdiag(j)
                if j >= 3 and pres[j]:
                    h = h + 0.5 * c.g2e * Ej @ Ej
                if lat.boundary == "free_flux" and not pres[j]:
                    h = h + 0.5 * c.g2e * Ej @ Ej
            self.terms.append((1.0, "phys", ((s, h),)))
        # hopping
        for (x, mu, y) in lat.links():
            w = [(x, "psid", None)] + _U(x, mu, y) + [(y, "psi", None)]
            self._word_term(-c.t, w)
            self._word_term(-c.t, _dagger_word(w))
        # plaquettes
        for (x, al, be) in lat.plaquettes():
            xa = lat.neighbour(x, 3 + al)
            xb = lat.neighbour(x, 3 + be)
            xab = lat.neighbour(xa, 3 + be)
            w = _U(x, al, xa) + _U(xa, be, xab) + _Udag(xb, al, xab) + _Udag(x, be, xb)
            self._word_term(-0.5 * c.g2m, w)
            self._word_term(-0.5 * c.g2m, _dagger_word(w))
        # link penalty: 1 - sum_a P^a(x,+mu) P^(2-a)(y,-mu)
        for (x, mu, y) in lat.links():
            self.offset["pen"] += 1.0
            for a in range(3):
                ops = (
                    (x, self.site_ops[x].proj(3 + mu, a)),
                    (y, self.site_ops[y].proj(mu, 2 - a)),
                )
                self.terms.append((-1.0, "pen", ops))

    def site_charges(self, s):
        return self.rows[s][:, 0] - self.lat.parity(s)
