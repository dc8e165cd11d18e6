"""Binary tree tensor network ground-state search (Methods, "Tensor
Networks"), plain dense-with-charge-labels form.

Tree (Methods, "Tensor Networks", 3D construction): bottom nodes merge two
neighbouring sites along x, the next layer merges along y, then z, and the
cycle repeats (an axis is skipped once a block spans the lattice along it).
Every node has three legs: children (l = lower block, r = upper block along
the merge axis) and parent p.  The root's parent leg has dimension one and
carries the total charge Q (the tree is made of three-leg tensors only).
Nodes are numbered layer by layer, within a layer in lexicographic (z, y, x)
order of their block origin; that is also the sweep order (lowest layer to
highest, one single-tensor update per node).

Link numbering: site s is link s (physical leg); node n's parent leg is
link N + n.

Sector allocation (the paper initialises the sector distribution randomly;
a deterministic rule is used so that two implementations can agree):
  * exact dimension per charge of a link from the subtree side, dS(q), and
    from the complement side, dC(Q - q) (product-space counts, saturated at
    2^62); a charge is allowed if both are > 0; cap(q) = min(dS, dC).
  * if sum cap <= chi the link is exact, else chi is split in proportion to
    W(q) = round(2^30 * w(q) / max w),  w(q) = pS(q) * pC(Q - q), where pS,
    pC are charge distributions of uniformly drawn product states (float64
    convolutions, ascending charge order, left operand = subtree first /
    complement first); integer largest-remainder split, ties broken by
    |q N - Q |S|| then by q; charges whose share reaches their cap are
    frozen at the cap and the rest re-split (water filling).
  * consistency: every sector of a leg must fit in the rows of any QR that
    isometrises a node toward that leg,
        n_p(q) <= sum_{q1} n_l(q1) n_r(q - q1),
        n_l(q) <= sum_{qr} n_r(qr) n_p(q + qr),  (and r likewise),
    enforced by repeated min-passes; empty sectors are dropped.

Update of a node (steps (i)-(iii)): H_eff from the environments, lowest
eigenpair by Lanczos started from the current node, node := Ritz vector.
The isometry centre moves between nodes along tree paths; each move is a
per-sector QR of the centre matricised against the leg it moves through
(diag(R) >= 0), R absorbed into the neighbour, and the environment of
that leg renormalised with the new isometry.

Environments of a link, from either side, hold block Hamiltonians of the
terms inside that side (one per class: "phys", "pen") and the open part of
every term that straddles the link.

Subspace expansion (Methods: single-tensor optimisation with subspace
expansion, which lets bond dimensions grow and symmetry sectors adapt; the
paper gives no formulas, the reading is this one).  On the first move after
a node a is updated, from a to its neighbour b across link e (a's leg w):
  1. e is extended: every charge Q that a's other legs can carry gets
     n+(Q) = min(n(Q) + delta, rows_a(Q)) columns (never fewer than n(Q)),
     the old ones first; a and b are zero-padded to the extended leg.
  2. Z = sum_k c_k (A_k (x) B_k (x) Omega_k) a+, over the terms k of a's
     H_eff that reach across e (factors A_k, B_k on a's other legs, None =
     identity), with Omega_k a random operator on the extended leg carrying
     the term's charge shift, nonzero only from old columns into padded
     ones (entries uniform in [-1, 1), counter-based generator, stream
     65536 * (expansion count) + term index, in the canonical operator
     layout).  Z lives in the padded columns only.
  3. M = a+ + alpha (|a+| / |Z|) Z; the state is unchanged because b+ has
     zero rows there.
  4. Per sector of the extended leg, M matricised against w is M = U S V^T.
     The largest singular values over all sectors are kept, at most chi_max
     of them and none below 1e-12 of the largest; the leg becomes the kept
     counts (empty sectors dropped), a := U_keep, b := (U_keep^T M) b+
     (= S_keep V_keep^T b+).
  5. The environment of e from a's side is rebuilt; the one from b's side
     is rebuilt when the centre next crosses e back.
With expansion on, every other move of the centre is the same SVD move
without steps 1-3: it drops zero singular values (and truncates to
chi_max), so a leg never keeps more columns than the rows behind it, which
the QR move would require.
"""

import math

import numpy as np

from .blocks import leg_charges, leg_dim
from .heff import mode_l, mode_p, mode_r
from .lanczos import lowest

SAT = 1 << 62
M64 = (1 << 64) - 1


def _splitmix(z):
    """SplitMix64 finaliser (Steele, Lea and Flood, 2014)."""
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix_sym_uniform(seed, stream, n):
    """n uniforms in [-1, 1) of the counter-based SplitMix64 stream
    (seed, stream): key = mix(seed ^ mix(stream + 0x632BE59BD9B4E019)),
    word_i = mix(key + (i + 1) * 0x9E3779B97F4A7C15), u = (word >> 11) 2^-53."""
    key = _splitmix((seed ^ _splitmix((stream + 0x632BE59BD9B4E019) & M64)) & M64)
    out = np.empty(n)
    for i in range(n):
        w = _splitmix((key + (i + 1) * 0x9E3779B97F4A7C15) & M64)
        out[i] = 2.0 * ((w >> 11) * 2.0 ** -53) - 1.0
    return out


# ----------------------------------------------------------------------
# tree geometry
# ----------------------------------------------------------------------
class Tree:
    def __init__(self, lat):
        self.lat = lat
        N = lat.nsites
        self.N = N
        if N < 2:
            raise ValueError("need at least two sites")
        for Lx in lat.L:
            if Lx & (Lx - 1):
                raise ValueError("lattice extents must be powers of two")
        blocks = [dict(origin=c, size=(1, 1, 1), link=lat.index(c))
                  for c in lat.iter_coords()]
        self.nodes = []
        self.sites_of = {s: frozenset([s]) for s in range(N)}
        axis, layer = 0, 0
        while len(blocks) > 1:
            for _ in range(3):
                if blocks[0]["size"][axis] < lat.L[axis]:
                    break
                axis = (axis + 1) % 3
            a = axis
            byorig = {b["origin"]: b for b in blocks}
            newb = []
            for b in blocks:
                o, sz = b["origin"], b["size"]
                if o[a] % (2 * sz[a]):
                    continue
                o2 = list(o); o2[a] += sz[a]
                b2 = byorig[tuple(o2)]
                nid = len(self.nodes)
                link = N + nid
                self.nodes.append(dict(l=b["link"], r=b2["link"], p=link,
                                       layer=layer, origin=o, axis=a))
                self.sites_of[link] = self.sites_of[b["link"]] | self.sites_of[b2["link"]]
                nsz = list(sz); nsz[a] *= 2
                newb.append(dict(origin=o, size=tuple(nsz), link=link))
            newb.sort(key=lambda b: (b["origin"][2], b["origin"][1], b["origin"][0]))
            blocks = newb
            axis = (a + 1) % 3
            layer += 1
        self.root = len(self.nodes) - 1
        self.top = N + self.root
        self.nlinks = N + len(self.nodes)
        # node owning each link as a child leg, and the side (0 = l, 1 = r)
        self.up = {}
        for n, nd in enumerate(self.nodes):
            self.up[nd["l"]] = (n, 0)
            self.up[nd["r"]] = (n, 1)
        self.all_sites = frozenset(range(N))

    def node_of_link(self, link):
        """Node whose parent leg is `link` (None for a site link)."""
        return link - self.N if link >= self.N else None

    def path(self, a, b):
        """Node path a -> b (inclusive) through the tree."""
        def anc(n):
            out = [n]
            while n != self.root:
                n = self.up[self.nodes[n]["p"]][0]
                out.append(n)
            return out
        pa, pb = anc(a), anc(b)
        sb = set(pb)
        lca = next(n for n in pa if n in sb)
        up = pa[: pa.index(lca) + 1]
        down = pb[: pb.index(lca)]
        return up + down[::-1]


# ----------------------------------------------------------------------
# sector allocation
# ----------------------------------------------------------------------
def _conv_int(a, b):
    out = {}
    for q1 in sorted(a):
        for q2 in sorted(b):
            v = min(SAT, a[q1] * b[q2])
            out[q1 + q2] = min(SAT, out.get(q1 + q2, 0) + v)
    return out


def _conv_float(a, b):
    keys = sorted({q1 + q2 for q1 in a for q2 in b})
    out = {}
    for q in keys:
        acc = 0.0
        for q1 in sorted(a):
            if q - q1 in b:
                acc = acc + a[q1] * b[q - q1]
        out[q] = acc
    return out


def link_distributions(tree, site_counts):
    """(dS, pS, dC, pC) per link: exact saturated counts and float
    distributions, subtree side and complement side."""
    dS, pS = {}, {}
    for s in range(tree.N):
        cnt = site_counts[s]
        tot = sum(cnt.values())
        dS[s] = dict(cnt)
        pS[s] = {q: c / tot for q, c in sorted(cnt.items())}
    for n, nd in enumerate(tree.nodes):
        dS[nd["p"]] = _conv_int(dS[nd["l"]], dS[nd["r"]])
        pS[nd["p"]] = _conv_float(pS[nd["l"]], pS[nd["r"]])
    dC = {tree.top: {0: 1}}
    pC = {tree.top: {0: 1.0}}
    for n in reversed(range(len(tree.nodes))):
        nd = tree.nodes[n]
        dC[nd["l"]] = _conv_int(dC[nd["p"]], dS[nd["r"]])
        pC[nd["l"]] = _conv_float(pC[nd["p"]], pS[nd["r"]])
        dC[nd["r"]] = _conv_int(dC[nd["p"]], dS[nd["l"]])
        pC[nd["r"]] = _conv_float(pC[nd["p"]], pS[nd["l"]])
    return dS, pS, dC, pC


def _split(budget, qs, W, cap, key):
    """Water-filling integer split of `budget` over charges qs."""
    n = {}
    free = [q for q in qs if cap[q] > 0 and W[q] > 0]
    while free and budget > 0:
        wsum = sum(W[q] for q in free)
        alloc = {q: (budget * W[q]) // wsum for q in free}
        rem = {q: (budget * W[q]) % wsum for q in free}
        left = budget - sum(alloc.values())
        for q in sorted(free, key=lambda q: (-rem[q],) + key(q))[:left]:
            alloc[q] += 1
        over = [q for q in free if alloc[q] >= cap[q]]
        if not over:
            n.update(alloc)
            break
        for q in over:
            n[q] = cap[q]
            budget -= cap[q]
            free.remove(q)
    return {q: v for q, v in n.items() if v > 0}


def allocate_sectors(tree, site_counts, Q, chi):
    """Leg sectors [(q, n)] for every link."""
    dS, pS, dC, pC = link_distributions(tree, site_counts)
    N = tree.N
    legs = {}
    for s in range(N):
        legs[s] = sorted(site_counts[s].items())
    legs[tree.top] = [(Q, 1)]
    for n, nd in enumerate(tree.nodes):
        e = nd["p"]
        if e == tree.top:
            continue
        qs = sorted(q for q in dS[e] if dS[e][q] > 0 and dC[e].get(Q - q, 0) > 0)
        cap = {q: min(dS[e][q], dC[e][Q - q]) for q in qs}
        if sum(cap.values()) <= chi:
            legs[e] = [(q, cap[q]) for q in qs]
            continue
        w = {q: pS[e][q] * pC[e][Q - q] for q in qs}
        wmax = max(w.values())
        W = {q: int(math.floor(w[q] / wmax * float(1 << 30) + 0.5)) for q in qs}
        size = len(tree.sites_of[e])

        def key(q, size=size):
            return (abs(q * N - Q * size), q)

        alloc = _split(chi, qs, W, cap, key)
        legs[e] = [(q, alloc[q]) for q in sorted(alloc)]
    _make_consistent(tree, legs)
    return legs


def _make_consistent(tree, legs):
    changed = True
    while changed:
        changed = False
        for nd in tree.nodes:
            L, R, P = (dict(legs[nd[k]]) for k in ("l", "r", "p"))
            # rows available for each sector of each leg
            newP = {q: min(n, sum(L[a] * R.get(q - a, 0) for a in L)) for q, n in P.items()}
            newL = {q: min(n, sum(R[b] * P.get(q + b, 0) for b in R)) for q, n in L.items()}
            newR = {q: min(n, sum(L[a] * P.get(q + a, 0) for a in L)) for q, n in R.items()}
            for k, new in (("l", newL), ("r", newR), ("p", newP)):
                if nd[k] < tree.N:
                    continue  # physical legs are never truncated
                leg = [(q, v) for q, v in sorted(new.items()) if v > 0]
                if leg != legs[nd[k]]:
                    legs[nd[k]] = leg
                    changed = True


# ----------------------------------------------------------------------
# environments
# ----------------------------------------------------------------------
class Env:
    """Operators of one side of a link in the basis of that link."""

    def __init__(self, chi):
        self.H = {"phys": np.zeros((chi, chi)), "pen": np.zeros((chi, chi))}
        self.open = {}


def renorm(n, which, A, B):
    """n^T (A (x) B) n contracted over the two legs other than `which`.
    A, B act on the remaining legs in order (l, r, p) minus `which`;
    None means identity.  Returns the operator on leg `which`
    (out[x, y] = sum n[.., x, ..] (A (x) B n)[.., y, ..])."""
    t = n
    if which == "p":
        if A is not None:
            t = mode_l(A, t)
        if B is not None:
            t = mode_r(B, t)
        return np.tensordot(n, t, axes=([0, 1], [0, 1]))
    if which == "l":
        if A is not None:
            t = mode_r(A, t)
        if B is not None:
            t = mode_p(B, t)
        return np.tensordot(n, t, axes=([1, 2], [1, 2]))
    if which == "r":
        if A is not None:
            t = mode_l(A, t)
        if B is not None:
            t = mode_p(B, t)
        return np.tensordot(n, t, axes=([0, 2], [0, 2]))
    raise ValueError(which)


# ----------------------------------------------------------------------
# the TTN state and its sweep
# ----------------------------------------------------------------------
class TTN:
    def __init__(self, ham, Q, chi, init=None, legs=None):
        """init: {node: flat canonical block vector} (seeded inputs)."""
        from .blocks import to_dense
        self.ham, self.Q, self.chi = ham, Q, chi
        self.lat = ham.lat
        self.tree = Tree(self.lat)
        N = self.tree.N
        counts = []
        for s in range(N):
            q = ham.site_charges(s)
            vals, c = np.unique(q, return_counts=True)
            counts.append({int(a): int(b) for a, b in zip(vals, c)})
        self.legs = legs if legs is not None else allocate_sectors(self.tree, counts, Q, chi)
        self.qv = {e: leg_charges(leg) for e, leg in self.legs.items()}
        # terms: (coef, cls, {site: matrix})
        self.terms = [(c, cls, dict(ops)) for c, cls, ops in ham.terms]
        self.nodes = []
        for n, nd in enumerate(self.tree.nodes):
            l, r, p = (self.legs[nd[k]] for k in ("l", "r", "p"))
            flat = init[n] if init is not None else None
            if flat is None:
                raise ValueError("initial node tensors must be supplied")
            self.nodes.append(to_dense(np.asarray(flat, dtype=float), l, r, p))
        self.env_up = {}
        self.env_dn = {}
        self.centre = None
        self.energy = None
        self.nu = 0.0
        self.expand = None          # dict(alpha, delta, chi_max, seed) or None
        self.n_expand = 0
        self.last_updated = None

    # -- helpers -------------------------------------------------------
    def legs_of(self, n):
        nd = self.tree.nodes[n]
        return nd["l"], nd["r"], nd["p"]

    def mask(self, n):
        l, r, p = (self.qv[e] for e in self.legs_of(n))
        return (l[:, None, None] + r[None, :, None] - p[None, None, :]) == 0

    def _site_env(self, s):
        ham = self.ham
        env = Env(ham.dims[s])
        for i, (c, cls, ops) in enumerate(self.terms):
            if s not in ops:
                continue
            if len(ops) == 1:
                env.H[cls] = env.H[cls] + c * ops[s]
            else:
                env.open[i] = ops[s]
        return env

    def _sides(self, n):
        """Site sets of the three sides of node n: (S_l, S_r, S_p)."""
        l, r, p = self.legs_of(n)
        Sl, Sr = self.tree.sites_of[l], self.tree.sites_of[r]
        return Sl, Sr, self.tree.all_sites - Sl - Sr

    def _env_for(self, n, which):
        """Environment of leg `which` of node n seen from outside n."""
        l, r, p = self.legs_of(n)
        if which == "l":
            return self.env_up[l]
        if which == "r":
            return self.env_up[r]
        return self.env_dn[p]

    # -- environment renormalisation ----------------------------------
    def _build_env(self, n, which):
        """Environment of leg `which` of node n, from the side opposite to
        where that leg points, using node n (an isometry toward `which`)."""
        sides = dict(zip("lrp", self._sides(n)))
        others = [k for k in "lrp" if k != which]
        e1, e2 = (self._env_for(n, k) for k in others)
        S1, S2 = sides[others[0]], sides[others[1]]
        S = S1 | S2
        node = self.nodes[n]
        chi = node.shape["lrp".index(which)]
        out = Env(chi)
        for cls in ("phys", "pen"):
            acc = renorm(node, which, e1.H[cls], None) + renorm(node, which, None, e2.H[cls])
            for i, (c, tcls, ops) in enumerate(self.terms):
                if tcls != cls:
                    continue
                st = set(ops)
                if st <= S and st & S1 and st & S2:
                    acc = acc + c * renorm(node, which, e1.open[i], e2.open[i])
            out.H[cls] = acc
        for i, (c, tcls, ops) in enumerate(self.terms):
            st = set(ops)
            if st & S and not st <= S:
                a = e1.open.get(i) if st & S1 else None
                b = e2.open.get(i) if st & S2 else None
                out.open[i] = renorm(node, which, a, b)
        return out

    # -- QR moves ------------------------------------------------------
    def _qr_toward(self, n, which):
        """Isometrise node n toward leg `which` per sector; return R as a
        dense chi x chi block-diagonal matrix (R[new, old])."""
        node = self.nodes[n]
        ax = "lrp".index(which)
        legs = self.legs_of(n)
        qv = [self.qv[e] for e in legs]
        mask = self.mask(n)
        moved = np.moveaxis(node, ax, -1)
        mmask = np.moveaxis(mask, ax, -1)
        qcol = qv[ax]
        chi = node.shape[ax]
        R = np.zeros((chi, chi))
        newm = np.zeros_like(moved)
        for q in np.unique(qcol):
            cols = np.nonzero(qcol == q)[0]
            rows = mmask[..., cols[0]]
            M = moved[rows][:, cols]
            if M.shape[0] < M.shape[1]:
                raise AssertionError("sector wider than its rows")
            Qm, Rm = np.linalg.qr(M, mode="reduced")
            sg = np.where(np.diag(Rm) < 0, -1.0, 1.0)
            Qm = Qm * sg[None, :]
            Rm = Rm * sg[:, None]
            sub = newm[rows]
            sub[:, cols] = Qm
            newm[rows] = sub
            R[np.ix_(cols, cols)] = Rm
        self.nodes[n] = np.moveaxis(newm, -1, ax)
        return R

    def _move(self, a, b):
        """Move the isometry centre from node a to its neighbour b."""
        ta, tb = self.tree.nodes[a], self.tree.nodes[b]
        if tb["l"] == ta["p"] or tb["r"] == ta["p"]:
            # up: isometrise a toward p, absorb R into b's child leg
            R = self._qr_toward(a, "p")
            side = "l" if tb["l"] == ta["p"] else "r"
            if side == "l":
                self.nodes[b] = np.einsum("xa,abc->xbc", R, self.nodes[b])
            else:
                self.nodes[b] = np.einsum("xb,abc->axc", R, self.nodes[b])
            self.env_up[ta["p"]] = self._build_env(a, "p")
        else:
            side = "l" if ta["l"] == tb["p"] else "r"
            R = self._qr_toward(a, side)
            self.nodes[b] = np.einsum("xc,abc->abx", R, self.nodes[b])
            link = ta[side]
            self.env_dn[link] = self._build_env(a, side)
        self.centre = b

    def move_to(self, target):
        path = self.tree.path(self.centre, target)
        for a, b in zip(path[:-1], path[1:]):
            if self.expand is not None:
                self._move_expand(a, b, grow=a == self.last_updated)
            else:
                self._move(a, b)
            self.last_updated = None

    # -- subspace expansion (reading in the module docstring) ----------
    def set_expansion(self, alpha, delta, chi_max, seed):
        self.expand = dict(alpha=float(alpha), delta=int(delta), chi_max=int(chi_max),
                           seed=int(seed))

    def _site_shift(self, s, M):
        q = self.ham.site_charges(s)
        x, y = np.nonzero(M)
        return int(q[x[0]] - q[y[0]])

    def _leg_shift(self, n, which, ops):
        """Charge shift of a term's factor on leg `which` of node n: the
        shifts of its site operators inside the leg's subtree (for p: inside
        n's subtree)."""
        Sl, Sr, _ = self._sides(n)
        S = {"l": Sl, "r": Sr, "p": Sl | Sr}[which]
        return sum(self._site_shift(s, M) for s, M in ops.items() if s in S)

    def _rows(self, n, which):
        """Row count per charge of node n matricised against leg `which`,
        over all sector pairs of its other two legs."""
        legs = dict(zip("lrp", (self.legs[e] for e in self.legs_of(n))))
        o1, o2 = [k for k in "lrp" if k != which]
        rows = {}
        for q1, n1 in legs[o1]:
            for q2, n2 in legs[o2]:
                if which == "p":
                    Q = q1 + q2
                elif which == "l":
                    Q = q2 - q1          # (r, p): q_l = q_p - q_r
                else:
                    Q = q2 - q1          # (l, p): q_r = q_p - q_l
                rows[Q] = rows.get(Q, 0) + n1 * n2
        return rows

    @staticmethod
    def _pad(T, ax, old, new):
        """Zero-pad axis ax from leg `old` to leg `new` (old columns first
        in every sector)."""
        from .blocks import leg_offsets
        oo, no = leg_offsets(old), leg_offsets(new)
        shape = list(T.shape)
        shape[ax] = leg_dim(new)
        out = np.zeros(shape)
        for q, n in old:
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[ax] = slice(oo[q], oo[q] + n)
            dst[ax] = slice(no[q], no[q] + n)
            out[tuple(dst)] = T[tuple(src)]
        return out

    def _omega(self, leg, old, delta, stream):
        """Random operator on `leg` with charge shift `delta`, nonzero only
        from old columns into padded ones."""
        from .blocks import leg_offsets
        off = leg_offsets(leg)
        size = dict(leg)
        total, lay = 0, []
        for q, n in leg:                       # canonical layout: input sectors ascending
            if q + delta in size:
                lay.append((q, total))
                total += size[q + delta] * n
        vals = splitmix_sym_uniform(self.expand["seed"], stream, total)
        oldn = dict(old)
        D = np.zeros((leg_dim(leg), leg_dim(leg)))
        for q, o in lay:
            qo = q + delta
            ni, no_ = size[q], size[qo]
            blk = vals[o:o + no_ * ni].reshape(no_, ni).copy()
            blk[:oldn.get(qo, 0), :] = 0.0      # existing output columns
            blk[:, oldn.get(q, 0):] = 0.0       # padded input columns
            D[off[qo]:off[qo] + no_, off[q]:off[q] + ni] = blk
        return D

    def _move_expand(self, a, b, grow=True):
        cfg = self.expand
        ta, tb = self.tree.nodes[a], self.tree.nodes[b]
        if tb["l"] == ta["p"] or tb["r"] == ta["p"]:
            w, wb, link = "p", ("l" if tb["l"] == ta["p"] else "r"), ta["p"]
        else:
            w = "l" if ta["l"] == tb["p"] else "r"
            wb, link = "p", ta[w]
        ax, axb = "lrp".index(w), "lrp".index(wb)
        old = list(self.legs[link])
        ra = self._rows(a, w)
        oldn = dict(old)
        sizes = dict(oldn)
        if grow:
            for Q in sorted(ra):
                n = max(oldn.get(Q, 0), min(oldn.get(Q, 0) + cfg["delta"], ra[Q]))
                if n > 0:
                    sizes[Q] = n
        plus = sorted(sizes.items())
        aP = self._pad(self.nodes[a], ax, old, plus)
        bP = self._pad(self.nodes[b], axb, old, plus)
        self.legs[link] = plus
        self.qv[link] = leg_charges(plus)
        # Z over the terms of a's H_eff that reach across the link
        env = {k: self._env_for(a, k) for k in "lrp"} if grow else {}
        sides = dict(zip("lrp", self._sides(a)))
        Z = np.zeros_like(aP)
        for i, (c, cls, ops) in enumerate(self.terms if grow else []):
            st = set(ops)
            touched = {k: bool(st & sides[k]) for k in "lrp"}
            if not touched[w] or sum(touched.values()) < 2:
                continue
            coef = c * (self.nu if cls == "pen" else 1.0)
            Om = self._omega(plus, old, self._leg_shift(a, w, ops), 65536 * self.n_expand + i)
            fac = {k: (env[k].open[i] if touched[k] else None) for k in "lrp" if k != w}
            fac[w] = Om
            Z += coef * self._apply3(aP, fac["l"], fac["r"], fac["p"])
        nz = np.linalg.norm(Z)
        M = aP + (cfg["alpha"] * np.linalg.norm(aP) / nz) * Z if nz > 0 else aP
        # per-sector SVD of M matricised against w: M = U S V^T
        qv = {k: self.qv[e] for k, e in zip("lrp", self.legs_of(a))}
        mask = (qv["l"][:, None, None] + qv["r"][None, :, None] - qv["p"][None, None, :]) == 0
        moved = np.moveaxis(M, ax, -1)
        mmask = np.moveaxis(mask, ax, -1)
        qcol = self.qv[link]
        parts = []
        for q in np.unique(qcol):
            cols = np.nonzero(qcol == q)[0]
            rows = mmask[..., cols[0]]
            Mq = moved[rows][:, cols]
            U, S, _ = np.linalg.svd(Mq, full_matrices=False)
            parts.append((int(q), cols, rows, Mq, U, S))
        smax = max((p[5].max() for p in parts if p[5].size), default=0.0)
        cand = sorted(((S[j], q, j) for q, _, _, _, _, S in parts for j in range(len(S))
                       if S[j] > 1e-12 * smax), key=lambda t: -t[0])[:cfg["chi_max"]]
        keep = {}
        for _, q, j in cand:
            keep.setdefault(q, []).append(j)
        new = [(q, len(keep[q])) for q in sorted(keep)]
        from .blocks import leg_offsets
        noff = leg_offsets(new)
        dplus, dnew = leg_dim(plus), leg_dim(new)
        anew = np.zeros(moved.shape[:-1] + (dnew,))
        W = np.zeros((dnew, dplus))
        for q, cols, rows, Mq, U, S in parts:
            if q not in keep:
                continue
            js = sorted(keep[q], key=lambda j: -S[j])
            Uq = U[:, js]
            nc = noff[q] + np.arange(len(js))
            sub = anew[rows]
            sub[:, nc] = Uq
            anew[rows] = sub
            W[np.ix_(nc, cols)] = Uq.T @ Mq
        self.nodes[a] = np.moveaxis(anew, -1, ax)
        self.nodes[b] = np.moveaxis(np.tensordot(W, np.moveaxis(bP, axb, 0), axes=(1, 0)), 0, axb)
        self.legs[link] = new
        self.qv[link] = leg_charges(new)
        if w == "p":
            self.env_up[link] = self._build_env(a, "p")
            self.env_dn.pop(link, None)
        else:
            self.env_dn[link] = self._build_env(a, w)
            self.env_up.pop(link, None)
        if grow:
            self.n_expand += 1
        self.centre = b

    @staticmethod
    def _apply3(t, A, B, C):
        if A is not None:
            t = mode_l(A, t)
        if B is not None:
            t = mode_r(B, t)
        if C is not None:
            t = mode_p(C, t)
        return t

    # -- set-up --------------------------------------------------------
    def prepare(self):
        """Isometrise bottom-up (centre ends at the root), building every
        upward environment; the root's parent environment is empty."""
        for s in range(self.tree.N):
            self.env_up[s] = self._site_env(s)
        for n in range(len(self.tree.nodes)):
            if n != self.tree.root and self.expand is not None:
                # expansion mode: SVD moves throughout (they build the environment)
                self._move_expand(n, self.tree.up[self.tree.nodes[n]["p"]][0], grow=False)
                continue
            if n != self.tree.root:
                nd = self.tree.nodes[n]
                R = self._qr_toward(n, "p")
                b, side = self.tree.up[nd["p"]]
                if side == 0:
                    self.nodes[b] = np.einsum("xa,abc->xbc", R, self.nodes[b])
                else:
                    self.nodes[b] = np.einsum("xb,abc->axc", R, self.nodes[b])
                self.env_up[nd["p"]] = self._build_env(n, "p")
        self.env_dn[self.tree.top] = Env(1)
        self.centre = self.tree.root

    # -- H_eff and the update -----------------------------------------
    def heff_terms(self, n, nu):
        """(c, A, B, C) list of the node's effective Hamiltonian."""
        El, Er, Ep = (self._env_for(n, k) for k in "lrp")
        Sl, Sr, Sp = self._sides(n)
        terms = []
        for cls, w in (("phys", 1.0), ("pen", nu)):
            terms.append((w, El.H[cls], None, None))
            terms.append((w, None, Er.H[cls], None))
            terms.append((w, None, None, Ep.H[cls]))
        for i, (c, cls, ops) in enumerate(self.terms):
            st = set(ops)
            touched = [bool(st & Sl), bool(st & Sr), bool(st & Sp)]
            if sum(touched) < 2:
                continue
            w = c * (nu if cls == "pen" else 1.0)
            terms.append((w,
                          El.open[i] if touched[0] else None,
                          Er.open[i] if touched[1] else None,
                          Ep.open[i] if touched[2] else None))
        return terms

    def offset(self, nu):
        return self.ham.offset["phys"] + nu * self.ham.offset["pen"]

    def update(self, n, nu, m=30, cycles=1, tol=0.0):
        from .heff import apply_dense
        terms = self.heff_terms(n, nu)
        mask = self.mask(n)
        shape = self.nodes[n].shape

        def apply(v):
            xd = np.zeros(shape)
            xd[mask] = v
            return apply_dense(xd, terms)[mask]

        x0 = self.nodes[n][mask]
        theta, u, resid = lowest(apply, x0, m=m, tol=tol, max_cycles=cycles)
        xd = np.zeros(shape)
        xd[mask] = u
        self.nodes[n] = xd
        self.energy = theta + self.offset(nu)
        self.last_updated = n
        return self.energy

    def sweep(self, nu, m=30, cycles=1, tol=0.0):
        """One sweep: every node once, lowest layer first; returns the
        energy after the last (root) update."""
        self.nu = nu
        if self.centre is None:
            self.prepare()
        for n in range(len(self.tree.nodes)):
            self.move_to(n)
            self.update(n, nu, m=m, cycles=cycles, tol=tol)
        return self.energy

    # -- observables ---------------------------------------------------
    def site_density_matrices(self):
        """rho for every site leg, top-down, with the centre at the root."""
        self.move_to(self.tree.root)
        rho = {self.tree.top: np.ones((1, 1))}
        root = self.nodes[self.tree.root]
        rho[self.tree.top] = np.ones((1, 1)) / np.einsum("abc,abc->", root, root)
        for n in reversed(range(len(self.tree.nodes))):
            nd = self.tree.nodes[n]
            x = self.nodes[n]
            rp = rho[nd["p"]]
            rho[nd["l"]] = np.einsum("abc,cd,xbd->ax", x, rp, x, optimize=True)
            rho[nd["r"]] = np.einsum("abc,cd,axd->bx", x, rp, x, optimize=True)
        return {s: rho[s] for s in range(self.tree.N)}

    def observables(self):
        """Per-site <phi>, per-(site, half-link) <k>, link field <E>,
        delta_L = sum_links |<L - 2>|, rho (matter density, reading
        n_x = (1 - (-1)^x)/2 + (-1)^x phi_x), total <Q>."""
        lat, ham = self.lat, self.ham
        rhos = self.site_density_matrices()
        N = lat.nsites
        phi = np.zeros(N)
        kexp = np.zeros((N, 6))
        for s in range(N):
            dg = np.diag(rhos[s])
            rows = ham.rows[s]
            phi[s] = dg @ rows[:, 0]
            kexp[s] = dg @ rows[:, 1:]
        efield = np.zeros((N, 3))
        dL = 0.0
        for (x, mu, y) in lat.links():
            efield[x, mu] = 1.0 - kexp[x, 3 + mu]
            dL += abs(kexp[x, 3 + mu] + kexp[y, mu] - 2.0)
        par = np.array([lat.parity(s) for s in range(N)])
        nocc = par + (1 - 2 * par) * phi
        return dict(phi=phi, k=kexp, efield=efield, deltaL=dL,
                    rho=float(nocc.mean()), Q=float((phi - par).sum()))


def penalty_schedule(s, nu_max, n_lin=4, n_quad=4):
    """nu for sweep s (Methods, "Numerical Convergence": linear growth,
    then quadratic growth, then constant at nu_max).  Constants are a
    reading: linear from nu_max/20 to nu_max/4 over n_lin sweeps, then
    quadratic to nu_max over n_quad sweeps."""
    lo, mid = nu_max / 20.0, nu_max / 4.0
    if s < n_lin:
        if n_lin == 1:
            return mid
        return lo + (mid - lo) * s / (n_lin - 1)
    if s < n_lin + n_quad:
        u = (s - n_lin + 1) / n_quad
        return mid + (nu_max - mid) * u * u
    return nu_max


def adaptive_penalty_schedule(s, energies, nu_max, n_lin=4, n_quad=4, rise=1e-10):
    """nu for sweep s under the adaptive switch (Methods, "Numerical
    Convergence": the penalty grows linearly until the energy is seen to
    rise slightly, then quadratically).  Reading: the linear phase has the
    slope of `penalty_schedule`; it ends after the first linear sweep t >= 1
    whose energy exceeds that of sweep t - 1 by more than rise |E_t| (or
    after n_lin sweeps); the quadratic phase then runs over n_quad sweeps
    from the nu of that last linear sweep to nu_max, and nu stays at nu_max
    afterwards.  energies[t] is the energy reported by sweep t; only sweeps
    before s are looked at."""
    lo, mid = nu_max / 20.0, nu_max / 4.0

    def linear(t):
        if n_lin == 1:
            return mid
        return lo + (mid - lo) * t / (n_lin - 1)

    switch = n_lin
    for t in range(1, min(n_lin, len(energies), s)):
        if energies[t] > energies[t - 1] + rise * abs(energies[t]):
            switch = t + 1
            break
    if s < switch:
        return linear(s)
    start = linear(switch - 1) if switch > 0 else mid
    k = s - switch
    if k < n_quad:
        u = (k + 1) / n_quad
        return start + (nu_max - start) * u * u
    return nu_max


def default_nu_max(cpl):
    """nu_max = 10 max(|t|, |m|, g_e^2/2, g_m^2/2) (a reading of the
    'much larger than the couplings' condition)."""
    return 10.0 * max(abs(cpl.t), abs(cpl.m), 0.5 * cpl.g2e, 0.5 * cpl.g2m)
