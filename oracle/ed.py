"""Exact diagonalisation on tiny lattices, two independent formulations.

(1) Original formulation (Results, "The model"): staggered fermions psi_x
    (Jordan-Wigner over the flat site order) and spin-1 links with
    E = S^z in {-1, 0, 1}, U raising E by one.  Physical states obey
    Gauss's law G_x = 0 (Gauss-law equation) with the outgoing-flux sign
    convention E_{x+mu,-mu} = -E_{x,mu}.  U has unit ladder elements (the
    link-state action printed in the Methods); `ladder="spin"` switches to
    U = S^+/s with s = 1 (elements sqrt(2)) as written in the QLM paragraph.
    Free-flux boundaries add one dangling flux variable per boundary
    half-link, with energy (g_e^2/2) E^2 and outgoing sign.
(2) Dressed-site formulation: product basis of the site bases, the term
    list of `hamiltonian.Hamiltonian`, optionally restricted to rishon
    number L = 2 on every link (then the penalty vanishes identically).

The two must give the same spectrum; this pins every fermionic sign of
the dressed-site operators.
"""

from itertools import product

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------
# (1) original formulation
# ----------------------------------------------------------------------
class OriginalED:
    def __init__(self, lat, cpl, Q=0, ladder="unit", dangling=None):
        self.lat, self.cpl, self.Q = lat, cpl, Q
        # optional {(site, half): E} pinning dangling fluxes (conserved)
        self.fix = dangling or {}
        self.amp = 1.0 if ladder == "unit" else np.sqrt(2.0)
        self.links = lat.links()
        self.lidx = {(x, mu): i for i, (x, mu, y) in enumerate(self.links)}
        self.dangling = []
        if lat.boundary == "free_flux":
            for s in range(lat.nsites):
                for j, pres in enumerate(lat.present(s)):
                    if not pres:
                        self.dangling.append((s, j))
        self._enumerate()
        self.H = self._build()

    def _enumerate(self):
        lat = self.lat
        nl, nd, N = len(self.links), len(self.dangling), lat.nsites
        par = np.array([lat.parity(s) for s in range(N)])
        # pinned dangling fluxes are substituted before expansion
        choices = [(-1, 0, 1)] * nl + [
            (self.fix[sj],) if sj in self.fix else (-1, 0, 1)
            for sj in self.dangling
        ]
        nfree = sum(len(c) > 1 for c in choices)
        if 3 ** nfree > 2_000_000:
            raise ValueError("lattice too large for the original-formulation ED")
        vals = np.array(list(product(*choices)), dtype=np.int64)
        vals = vals.reshape(-1, nl + nd)
        div = np.zeros((vals.shape[0], N), dtype=np.int64)
        for i, (x, mu, y) in enumerate(self.links):
            div[:, x] += vals[:, i]
            div[:, y] -= vals[:, i]
        for i, (s, j) in enumerate(self.dangling):
            div[:, s] += vals[:, nl + i]
        phi = par[None, :] + div
        ok = np.all((phi >= 0) & (phi <= 1), axis=1)
        ok &= (phi - par[None, :]).sum(axis=1) == self.Q
        self.E = vals[ok]
        self.phi = phi[ok]
        self.index = {
            (tuple(p), tuple(e)): i for i, (p, e) in enumerate(zip(self.phi, self.E))
        }
        self.dim = len(self.index)

    def _build(self):
        lat, c = self.lat, self.cpl
        nl = len(self.links)
        rows, cols, vals = [], [], []
        sgn = np.array([1 - 2 * lat.parity(s) for s in range(lat.nsites)])
        plaqs = []
        for (x, al, be) in lat.plaquettes():
            xa = lat.neighbour(x, 3 + al)
            xb = lat.neighbour(x, 3 + be)
            plaqs.append(
                (self.lidx[(x, al)], self.lidx[(xa, be)],
                 self.lidx[(xb, al)], self.lidx[(x, be)])
            )
        for i in range(self.dim):
            phi, E = self.phi[i], self.E[i]
            diag = c.m * float(np.dot(sgn, phi)) + 0.5 * c.g2e * float(np.dot(E, E))
            if c.mu:
                diag += float(np.dot(np.asarray(c.mu, dtype=float), phi))
            rows.append(i); cols.append(i); vals.append(diag)
            # hopping psi^dag_x U psi_y and its conjugate
            for li, (x, mu, y) in enumerate(self.links):
                if phi[x] == 0 and phi[y] == 1 and E[li] < 1:
                    s1 = (-1) ** int(phi[:y].sum())
                    p2 = phi.copy(); p2[y] = 0
                    s2 = (-1) ** int(p2[:x].sum())
                    p2[x] = 1
                    E2 = E.copy(); E2[li] += 1
                    j = self.index[(tuple(p2), tuple(E2))]
                    v = -c.t * self.amp * s1 * s2
                    rows += [j, i]; cols += [i, j]; vals += [v, v]
            # plaquette box and its conjugate
            for (l1, l2, l3, l4) in plaqs:
                if E[l1] < 1 and E[l2] < 1 and E[l3] > -1 and E[l4] > -1:
                    E2 = E.copy()
                    E2[l1] += 1; E2[l2] += 1; E2[l3] -= 1; E2[l4] -= 1
                    j = self.index[(tuple(phi), tuple(E2))]
                    v = -0.5 * c.g2m * self.amp ** 4
                    rows += [j, i]; cols += [i, j]; vals += [v, v]
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))

    def spectrum(self, k=None):
        H = self.H.toarray()
        w = np.linalg.eigvalsh(H)
        return w if k is None else w[:k]


# ----------------------------------------------------------------------
# (2) dressed-site formulation
# ----------------------------------------------------------------------
def _sparse_cols(M, tol=0.0):
    """Column-wise nonzeros of a dense matrix: list over columns of
    [(row, value)]."""
    out = []
    for j in range(M.shape[1]):
        nz = np.nonzero(np.abs(M[:, j]) > tol)[0]
        out.append([(int(i), float(M[i, j])) for i in nz])
    return out


class DressedED:
    """Product basis of dressed sites with total charge Q; `link2=True`
    keeps only states with rishon number 2 on every link."""

    def __init__(self, ham, Q=0, nu=0.0, link2=True, dangling=None):
        self.ham, self.Q, self.nu, self.link2 = ham, Q, nu, link2
        # optional {(site, half): E} pinning dangling fluxes, E = 1 - k
        self.fix = dangling or {}
        lat = ham.lat
        self.links = lat.links()
        self._enumerate()
        self.H = self._build()

    def _enumerate(self):
        ham, lat = self.ham, self.ham.lat
        N = lat.nsites
        q = [ham.site_charges(s) for s in range(N)]
        rows = ham.rows
        # links checked when their upper site is assigned (sites in order)
        lower_links = {s: [] for s in range(N)}
        for (x, mu, y) in self.links:
            lower_links[max(x, y)].append((x, mu, y))
        qmin = [min(v) for v in q]
        qmax = [max(v) for v in q]
        states = []

        def rec(s, cur, qsum):
            if s == N:
                if qsum == self.Q:
                    states.append(tuple(cur))
                return
            rest_min = sum(qmin[s + 1:])
            rest_max = sum(qmax[s + 1:])
            for i in range(ham.dims[s]):
                if any(1 - rows[s][i][1 + j] != e
                       for (ss, j), e in self.fix.items() if ss == s):
                    continue
                qs = qsum + int(q[s][i])
                if not (rest_min <= self.Q - qs <= rest_max):
                    continue
                if self.link2:
                    good = True
                    for (x, mu, y) in lower_links[s]:
                        kx = rows[x][cur[x] if x < s else i][1 + 3 + mu]
                        ky = rows[y][cur[y] if y < s else i][1 + mu]
                        if kx + ky != 2:
                            good = False
                            break
                    if not good:
                        continue
                cur.append(i)
                rec(s + 1, cur, qs)
                cur.pop()

        rec(0, [], 0)
        self.states = states
        self.index = {st: i for i, st in enumerate(states)}
        self.dim = len(states)

    def _build(self):
        ham = self.ham
        rows, cols, vals = [], [], []
        terms = []
        for coef, cls, ops in ham.terms:
            c = coef * (self.nu if cls == "pen" else 1.0)
            if c == 0.0:
                continue
            terms.append((c, [(s, _sparse_cols(M)) for s, M in ops]))
        const = ham.offset["phys"] + self.nu * ham.offset["pen"]
        for i, st in enumerate(self.states):
            if const:
                rows.append(i); cols.append(i); vals.append(const)
            for c, facs in terms:
                branches = [(list(st), c)]
                for s, colnz in facs:
                    nb = []
                    for cur, v in branches:
                        for (r, a) in colnz[cur[s]]:
                            nxt = list(cur); nxt[s] = r
                            nb.append((nxt, v * a))
                    branches = nb
                for cur, v in branches:
                    j = self.index.get(tuple(cur))
                    if j is None:
                        if self.link2:
                            raise AssertionError("term leaves the L=2 sector")
                        continue
                    rows.append(j); cols.append(i); vals.append(v)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))

    def spectrum(self, k=None):
        w = np.linalg.eigvalsh(self.H.toarray())
        return w if k is None else w[:k]


def dense_dressed_hamiltonian(ham, nu):
    """Full product-space operator (all charges) by Kronecker products;
    only for a handful of tiny sites."""
    N = ham.lat.nsites
    dims = ham.dims
    D = int(np.prod(dims))
    H = np.zeros((D, D))
    for coef, cls, ops in ham.terms:
        c = coef * (nu if cls == "pen" else 1.0)
        mats = [np.eye(dims[s]) for s in range(N)]
        for s, M in ops:
            mats[s] = M
        K = mats[0]
        for s in range(1, N):
            K = np.kron(K, mats[s])
        H += c * K
    H += (ham.offset["phys"] + nu * ham.offset["pen"]) * np.eye(D)
    return H


def product_charges(ham):
    """Total charge of every product basis state (kron order: site 0 is
    the slowest index)."""
    N = ham.lat.nsites
    q = np.zeros(1, dtype=np.int64)
    for s in range(N):
        q = (q[:, None] + ham.site_charges(s)[None, :]).reshape(-1)
    return q
