"""U(1) block structure of three-leg tree tensors (Methods, "Tensor
Networks": the TTN carries global U(1) symmetry sectors on every leg).

A leg is a list [(q, n)] of charges (strictly ascending) and sector sizes
(> 0).  A three-leg tensor with legs (l, r, p) and flux f keeps only the
blocks with  q_l + q_r - q_p = f  (a tree node has f = 0: the parent leg
carries the total charge of the two children).

Canonical layout (shared contract with the library, a reading since the
paper fixes none): blocks sorted by (q_l, q_r) ascending, a block kept
only if q_p = q_l + q_r - f is a sector of p; block b occupies
flat[off[b] : off[b+1]] with off the prefix sums of n_l n_r n_p, and the
in-block index is (i_l * n_r + i_r) * n_p + i_p.
"""

import numpy as np


def leg_dim(leg):
    return sum(n for _, n in leg)


def leg_offsets(leg):
    out, o = {}, 0
    for q, n in leg:
        out[q] = o
        o += n
    return out


def leg_charges(leg):
    """Charge of every index of the leg (dense order)."""
    return np.concatenate([np.full(n, q, dtype=np.int64) for q, n in leg]) \
        if leg else np.zeros(0, dtype=np.int64)


def block_table(l, r, p, flux=0):
    """[(il, ir, ip)] sector indices of the allowed blocks, canonical
    order, and int64 offsets (nblk + 1)."""
    pidx = {q: i for i, (q, _) in enumerate(p)}
    triples = []
    for il, (ql, nl) in enumerate(l):
        for ir, (qr, nr) in enumerate(r):
            qp = ql + qr - flux
            if qp in pidx:
                triples.append((il, ir, pidx[qp]))
    offs = [0]
    for il, ir, ip in triples:
        offs.append(offs[-1] + l[il][1] * r[ir][1] * p[ip][1])
    return triples, np.array(offs, dtype=np.int64)


def to_dense(flat, l, r, p, flux=0):
    triples, offs = block_table(l, r, p, flux)
    ol, orr, op = leg_offsets(l), leg_offsets(r), leg_offsets(p)
    D = np.zeros((leg_dim(l), leg_dim(r), leg_dim(p)))
    for b, (il, ir, ip) in enumerate(triples):
        (ql, nl), (qr, nr), (qp, np_) = l[il], r[ir], p[ip]
        blk = np.asarray(flat[offs[b]:offs[b + 1]]).reshape(nl, nr, np_)
        D[ol[ql]:ol[ql] + nl, orr[qr]:orr[qr] + nr, op[qp]:op[qp] + np_] = blk
    return D


def from_dense(D, l, r, p, flux=0):
    triples, offs = block_table(l, r, p, flux)
    ol, orr, op = leg_offsets(l), leg_offsets(r), leg_offsets(p)
    flat = np.zeros(int(offs[-1]))
    for b, (il, ir, ip) in enumerate(triples):
        (ql, nl), (qr, nr), (qp, np_) = l[il], r[ir], p[ip]
        blk = D[ol[ql]:ol[ql] + nl, orr[qr]:orr[qr] + nr, op[qp]:op[qp] + np_]
        flat[offs[b]:offs[b + 1]] = blk.reshape(-1)
    return flat


def allowed_mask(l, r, p, flux=0):
    ql, qr, qp = leg_charges(l), leg_charges(r), leg_charges(p)
    return (ql[:, None, None] + qr[None, :, None] - qp[None, None, :]) == flux


# -- operators on one leg ---------------------------------------------
def op_to_dense(blocks, leg, delta):
    """Block-sparse leg operator {q_in: (n_{q_in+delta} x n_{q_in})} with
    charge shift delta, embedded as a dense chi x chi matrix."""
    o = leg_offsets(leg)
    sizes = dict(leg)
    D = np.zeros((leg_dim(leg), leg_dim(leg)))
    for q, M in blocks.items():
        qo = q + delta
        if q not in sizes or qo not in sizes:
            continue
        D[o[qo]:o[qo] + sizes[qo], o[q]:o[q] + sizes[q]] = M
    return D


def op_from_dense(D, leg, delta):
    o = leg_offsets(leg)
    sizes = dict(leg)
    out = {}
    for q, n in leg:
        qo = q + delta
        if qo in sizes:
            out[q] = D[o[qo]:o[qo] + sizes[qo], o[q]:o[q] + n].copy()
    return out
