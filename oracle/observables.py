"""Observables of the paper's figures, computed from local expectation
values (test infrastructure: only the tests, the smoke check and the CPU
baseline of the benchmark use this package).

Local inputs are per site x:
    charge[x]  = <q_x>, the Gauss-law charge q_x = psi^dag psi - p_x with
                 p_x = (1 - (-1)^x)/2 (Results, "The model": charge and
                 Gauss's law);
    flux[x, h] = <outgoing electric flux on half-link h>, h in the order
                 -x, -y, -z, +x, +y, +z; on a +mu half-link it is E_{x,mu},
                 on a -mu half-link it is -E_{x-mu,mu}; a dangling
                 boundary half-link carries its own flux; a half-link with
                 no field (zero-flux boundary) carries 0.
Gauss's law reads sum_h flux[x, h] = charge[x] on every site.  The
fluxes of the two halves of a link cancel only in the physical subspace
(rishon number 2 on the link), so plane-summed relations hold exactly
there and, for a dressed-site state outside it, up to the link defects.

Profiles (Results, "Quantum capacitor" and "Finite density"):
    q_c(d)  = (2/A) sum over plane d of <q_x>,         d = 0 .. L_a - 1
    E^c(d)  = (2/A) sum over plane d-1 of <E_{x,a}>,   d = 0 .. L_a
              (E^c(0) / E^c(L_a) are the fluxes through the lower / upper
              face, zero under the zero-flux boundary),
    sigma(l) = mean of <q_x> over the sites whose distance to the closest
              boundary is l (l = 1 on the surface),
with A the number of sites of a plane orthogonal to axis a.  The charge
profile and the surface density use the Gauss-law charge q_x: the
paper's printed forms multiply psi^dag psi by the staggered sign, which
equals q_x in the convention where odd sites are hole-transformed; with
the convention used here (vacuum: even sites empty, odd sites filled) q_x
is what vanishes in the vacuum and reaches +-1 on charged plates.

Static potential (Results, "Confinement properties"): opposite static
charges are pinned by large local chemical potentials, and
V(r) = E(r) - E_0 up to an r-independent constant.
"""

import numpy as np


def ed_ground_state(ed):
    """Lowest eigenpair of an `ed.OriginalED` problem (dense eigh)."""
    w, v = np.linalg.eigh(ed.H.toarray())
    return w[0], v[:, 0], (w[1] - w[0]) if len(w) > 1 else np.inf


def ed_local_expectations(ed, vec):
    """(charge[N], flux[N, 6]) of a state of the original formulation.

    The ED basis stores, per basis state, the matter occupations phi_x and
    the link fields E_l (links (x, mu, y = x + mu)) followed by the dangling
    boundary fluxes (site, half-link), the latter in the outgoing sign."""
    lat = ed.lat
    N = lat.nsites
    prob = np.asarray(vec, dtype=np.float64) ** 2
    par = np.array([lat.parity(s) for s in range(N)], dtype=np.float64)
    charge = prob @ ed.phi.astype(np.float64) - par
    field = prob @ ed.E.astype(np.float64)
    flux = np.zeros((N, 6))
    for i, (x, mu, y) in enumerate(ed.links):
        flux[x, 3 + mu] += field[i]
        flux[y, mu] -= field[i]
    nl = len(ed.links)
    for j, (s, h) in enumerate(ed.dangling):
        flux[s, h] += field[nl + j]
    return charge, flux


def plane_profiles(dims, charge, flux, axis):
    """(q_c[L_a], E^c[L_a + 1]) along `axis`; see the module docstring."""
    dims = tuple(int(v) for v in dims)
    La = dims[axis]
    area = dims[0] * dims[1] * dims[2] // La
    qc = np.zeros(La)
    ec = np.zeros(La + 1)
    for s in range(dims[0] * dims[1] * dims[2]):
        c = (s % dims[0], (s // dims[0]) % dims[1], s // (dims[0] * dims[1]))
        d = c[axis]
        qc[d] += charge[s]
        # the +a half-link of plane d carries the field from plane d to d + 1
        ec[d + 1] += flux[s, 3 + axis]
        if d == 0:
            # field entering through the lower face along +a
            ec[0] -= flux[s, axis]
    return 2.0 * qc / area, 2.0 * ec / area


def shell_of(dims, s):
    """Distance of site s to the closest boundary, 1 on the surface."""
    c = (s % dims[0], (s // dims[0]) % dims[1], s // (dims[0] * dims[1]))
    return 1 + min(min(c[a], dims[a] - 1 - c[a]) for a in range(3))


def surface_density(dims, charge):
    """sigma(l) for l = 1 .. n_shell (Finite density, surface density eq.)."""
    dims = tuple(int(v) for v in dims)
    n = dims[0] * dims[1] * dims[2]
    shells = [shell_of(dims, s) for s in range(n)]
    nshell = max(shells)
    tot = np.zeros(nshell)
    cnt = np.zeros(nshell)
    for s in range(n):
        tot[shells[s] - 1] += charge[s]
        cnt[shells[s] - 1] += 1
    return tot / cnt


def pinning_potentials(dims, pins, lam):
    """Chemical potentials mu_x that pin static charges.

    pins: {site: q} with q in {-1, 0, +1}.  The onsite term mu_x psi^dag psi
    favours psi^dag psi = 1 for mu_x = -lam and 0 for mu_x = +lam; the
    charge q = psi^dag psi - p_x then fixes the occupation to pin:
    +1 needs an even site (filled), -1 an odd site (empty), 0 the vacuum
    occupation of the site's parity."""
    n = int(dims[0]) * int(dims[1]) * int(dims[2])
    mu = np.zeros(n)
    for s, q in pins.items():
        c = (s % dims[0], (s // dims[0]) % dims[1], s // (dims[0] * dims[1]))
        p = sum(c) % 2
        occ = q + p
        if occ not in (0, 1):
            raise ValueError(f"charge {q} cannot sit on a site of parity {p}")
        mu[s] = -lam if occ == 1 else lam
    return mu


def dressed_local_expectations(ded, vec):
    """(charge[N], flux[N, 6]) of a state of the dressed-site formulation
    (`ed.DressedED`): per site the Gauss-law charge phi - p and, on every
    half-link, the outgoing flux 1 - k (rishon number k; a frozen boundary
    half-link has k = 1)."""
    ham = ded.ham
    N = ham.lat.nsites
    prob = np.asarray(vec, dtype=np.float64) ** 2
    charge = np.zeros(N)
    flux = np.zeros((N, 6))
    for pr, st in zip(prob, ded.states):
        for s in range(N):
            row = ham.rows[s][st[s]]
            charge[s] += pr * (row[0] - ham.lat.parity(s))
            flux[s] += pr * (1.0 - row[1:7])
    return charge, flux
