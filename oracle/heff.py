"""Effective Hamiltonian of one tree node (Methods, "Tensor Networks",
step (i) of the single-tensor update): the full Hamiltonian contracted with
every other tensor of the tree leaves a sum of products of operators on the
node's three legs,
    H_eff = sum_k c_k  A_k (x) B_k (x) C_k        (A on l, B on r, C on p),
each factor either the identity or a renormalised operator with an integer
U(1) shift delta, delta_A + delta_B = delta_C.

`apply_dense` is the plain definition: embed the node tensor densely and
contract  y_ijk = sum_k c_k A_ia B_jb C_kc x_abc  (einsum).  `matrix`
builds the explicit |x| x |x| operator for tiny nodes.  `adjoint_dense`
is the reverse-mode derivative of <ybar, y> with respect to x, every
factor and every coefficient (the derivative of the energy with respect
to the node tensor and to the couplings, by the chain rule).  A term is
(c, A, B, C) with dense chi x chi matrices or None for the identity.
"""

import numpy as np

from .blocks import allowed_mask, block_table, from_dense, to_dense


def mode_l(A, t):
    """(A x_l t)_ijk = sum_a A_ia t_ajk"""
    return np.tensordot(A, t, axes=(1, 0))


def mode_r(B, t):
    """(B x_r t)_ijk = sum_b B_jb t_ibk"""
    return np.tensordot(B, t, axes=(1, 1)).transpose(1, 0, 2)


def mode_p(C, t):
    """(C x_p t)_ijk = sum_c C_kc t_ijc"""
    return np.tensordot(t, C, axes=(2, 1))


def apply_dense(xd, terms):
    y = np.zeros_like(xd)
    for c, A, B, C in terms:
        t = xd
        if A is not None:
            t = mode_l(A, t)
        if B is not None:
            t = mode_r(B, t)
        if C is not None:
            t = mode_p(C, t)
        y += c * t
    return y


def apply_flat(x, legs, terms):
    """Same operator on the canonical flat block vector."""
    l, r, p = legs
    y = apply_dense(to_dense(x, l, r, p), terms)
    # everything the operator produces must live on allowed blocks
    if np.abs(y[~allowed_mask(l, r, p)]).max(initial=0.0) > 0.0:
        raise AssertionError("H_eff leaked out of the allowed blocks")
    return from_dense(y, l, r, p)


def matrix(legs, terms):
    """Explicit matrix in the flat block basis (columns = H e_i)."""
    l, r, p = legs
    size = int(allowed_mask(l, r, p).sum())
    H = np.zeros((size, size))
    e = np.zeros(size)
    for i in range(size):
        e[:] = 0.0
        e[i] = 1.0
        H[:, i] = apply_flat(e, legs, terms)
    return H


def flops(legs, metas):
    """Algorithmic flop count of one application.

    metas: per term (hasA, dA, hasB, dB, hasC, dC) with dX the charge
    shift of factor X.  Each non-identity factor is applied to each
    allowed block as a dense mode product, in the order C (on p), then
    B (on r), then A (on l), each step on the extents the previous one
    produced; a term whose output block does not exist costs nothing;
    identity factors cost nothing.  Sector-preserving case:
    2 n_l n_r n_p (n_l + n_r + n_p) per block and three-factor term.
    """
    l, r, p = legs
    triples, _ = block_table(l, r, p)
    sl, sr, sp_ = dict(l), dict(r), dict(p)
    total = 0
    for hasA, dA, hasB, dB, hasC, dC in metas:
        for il, ir, ip in triples:
            ql, qr, qp = l[il][0], r[ir][0], p[ip][0]
            oq = (ql + (dA if hasA else 0), qr + (dB if hasB else 0),
                  qp + (dC if hasC else 0))
            if oq[0] not in sl or oq[1] not in sr or oq[2] not in sp_:
                continue
            na, nb, nc = sl[ql], sr[qr], sp_[qp]
            na2, nb2, nc2 = sl[oq[0]], sr[oq[1]], sp_[oq[2]]
            if hasC:
                total += 2 * na * nb * nc * nc2
            if hasB:
                total += 2 * na * nb * nb2 * nc2
            if hasA:
                total += 2 * na * na2 * nb2 * nc2
    return total


def adjoint_dense(xd, ybd, terms):
    """Reverse mode of y = apply_dense(x, terms) for the scalar <ybar, y>.

    Since y is linear in x, in every factor and in every coefficient, the
    derivatives follow from the definition term by term:
      xbar           = sum_k c_k (A_k^T x_l B_k^T x_r C_k^T x_p ybar)
      Abar_k[i, a]   = c_k sum_{j,k'} ybar[i,j,k'] (B_k x_r C_k x_p x)[a,j,k']
      Bbar_k[j, b]   = c_k sum_{i,k'} ybar[i,j,k'] (A_k x_l C_k x_p x)[i,b,k']
      Cbar_k[k', c]  = c_k sum_{i,j}  ybar[i,j,k'] (A_k x_l B_k x_r x)[i,j,c]
      cbar_k         = <ybar, A_k x_l B_k x_r C_k x_p x>
    Identity factors have no gradient (None).  Returns
    (xbar, [(Abar, Bbar, Cbar)], cbar) with dense arrays."""
    xbar = np.zeros_like(xd)
    grads, cbar = [], []
    for c, A, B, C in terms:
        t = ybd
        if A is not None:
            t = mode_l(A.T, t)
        if B is not None:
            t = mode_r(B.T, t)
        if C is not None:
            t = mode_p(C.T, t)
        xbar += c * t

        def part(skip):
            u = xd
            if A is not None and skip != 0:
                u = mode_l(A, u)
            if B is not None and skip != 1:
                u = mode_r(B, u)
            if C is not None and skip != 2:
                u = mode_p(C, u)
            return u

        g = [None, None, None]
        if A is not None:
            g[0] = c * np.einsum("ijk,ajk->ia", ybd, part(0))
        if B is not None:
            g[1] = c * np.einsum("ijk,ibk->jb", ybd, part(1))
        if C is not None:
            g[2] = c * np.einsum("ijk,ijc->kc", ybd, part(2))
        grads.append(tuple(g))
        cbar.append(float(np.sum(ybd * part(-1))))
    return xbar, grads, np.array(cbar)
