"""Site-local operators from an explicit fermionic Fock space.

Construction (Methods, "Fermionic compact representation ..."):
  * a dressed site carries 13 Dirac modes: the matter mode psi, then for
    each half-link j = 0..5 two modes a_j, b_j.  Mode order inside a site:
    psi, a_0, b_0, a_1, b_1, ..., a_5, b_5 (the paper lists psi first and
    the half-links in the basis order; any fixed order gives the same
    spectrum, and the exact-diagonalisation tests pin the result).
  * Fock states are built by applying creation-operator matrices
    (Jordan-Wigner within the site) to the vacuum.
  * the 3-hardcore rishon is eta_j^dag = n^a_j b_j^dag + (1 - n^b_j) a_j^dag
    (3-hardcore mode equation); half-link states |0>, |1> = a^dag|0>,
    |2> = b^dag a^dag |0>.
  * a dressed basis state (phi, k_1..k_6) is
        (-1)^(d(k1,2)+d(k2,2)+d(k3,2)) (psi^dag)^phi  K_1 ... K_6 |vac>
    with K_j the creation word of |k_j> (local basis equation).

Any product of an even number of mode operators is then a bosonic
site-local matrix; it is projected on the dressed basis with B^T O B,
and the projection is checked to be exact (no leakage out of the Gauss
subspace).
"""

from functools import lru_cache

import numpy as np
import scipy.sparse as sp

NMODES = 13
DIM = 1 << NMODES


def _mode_index(kind, j=None):
    if kind == "psi":
        return 0
    if kind == "a":
        return 1 + 2 * j
    if kind == "b":
        return 2 + 2 * j
    raise ValueError(kind)


@lru_cache(maxsize=None)
def annihilator(m, nmodes=NMODES):
    """c_m on the 2^nmodes Fock space, occupation basis, Jordan-Wigner
    order by mode index (bit m of the state integer = n_m)."""
    dim = 1 << nmodes
    rows, cols, vals = [], [], []
    for s in range(dim):
        if (s >> m) & 1:
            t = s & ~(1 << m)
            below = bin(s & ((1 << m) - 1)).count("1")
            rows.append(t)
            cols.append(s)
            vals.append(-1.0 if below % 2 else 1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def creator(m, nmodes=NMODES):
    return annihilator(m, nmodes).T.tocsr()


def number(m, nmodes=NMODES):
    return (creator(m, nmodes) @ annihilator(m, nmodes)).tocsr()


IDENT = sp.identity(DIM, format="csr")


def rishon_dag(ma, mb, nmodes=NMODES):
    """eta^dag = n^a b^dag + (1 - n^b) a^dag on modes (ma, mb)
    (3-hardcore mode equation)."""
    one = sp.identity(1 << nmodes, format="csr")
    return (number(ma, nmodes) @ creator(mb, nmodes)
            + (one - number(mb, nmodes)) @ creator(ma, nmodes)).tocsr()


@lru_cache(maxsize=None)
def eta_dag(j):
    """3-hardcore creation on half-link j of a dressed site."""
    return rishon_dag(_mode_index("a", j), _mode_index("b", j))


@lru_cache(maxsize=None)
def eta(j):
    return eta_dag(j).T.tocsr()


def psi():
    return annihilator(0)


def psi_dag():
    return creator(0)


def mode_op(kind, j=None):
    """Single odd operator: kind in psi, psid, eta, etad."""
    if kind == "psi":
        return psi()
    if kind == "psid":
        return psi_dag()
    if kind == "eta":
        return eta(j)
    if kind == "etad":
        return eta_dag(j)
    raise ValueError(kind)


def basis_vectors(rows):
    """DIM x d matrix whose columns are the dressed basis states."""
    vac = np.zeros(DIM)
    vac[0] = 1.0
    cols = []
    for r in rows:
        phi, ks = int(r[0]), [int(x) for x in r[1:]]
        v = vac.copy()
        # build right-to-left: the rightmost creation word acts first
        for j in reversed(range(6)):
            a = creator(_mode_index("a", j))
            b = creator(_mode_index("b", j))
            if ks[j] >= 1:
                v = a @ v
            if ks[j] == 2:
                v = b @ v
        if phi:
            v = psi_dag() @ v
        sign = (-1) ** (int(ks[0] == 2) + int(ks[1] == 2) + int(ks[2] == 2))
        cols.append(sign * v)
    return np.array(cols).T


class SiteOps:
    """Dressed-site matrices of words of mode operators for one basis."""

    def __init__(self, rows):
        self.rows = np.asarray(rows)
        self.B = sp.csr_matrix(basis_vectors(self.rows))
        self.d = self.rows.shape[0]

    def word(self, ops):
        """Matrix of the ordered product ops[0] @ ops[1] @ ... projected
        on the dressed basis; ops are (kind, j) pairs, even in number."""
        if len(ops) % 2:
            raise ValueError("odd word is not site-local")
        M = IDENT
        for kind, j in ops:
            M = M @ mode_op(kind, j)
        OB = M @ self.B
        R = (self.B.T @ OB).toarray()
        leak = OB - self.B @ sp.csr_matrix(R)
        if leak.nnz and abs(leak).max() > 1e-12:
            raise AssertionError("operator leaves the Gauss-law subspace")
        return R

    # convenient diagonal operators read straight off the basis rows
    def phi(self):
        return np.diag(self.rows[:, 0].astype(float))

    def kdiag(self, j):
        return np.diag(self.rows[:, 1 + j].astype(float))

    def proj(self, j, a):
        return np.diag((self.rows[:, 1 + j] == a).astype(float))
