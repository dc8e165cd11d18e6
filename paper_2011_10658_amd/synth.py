"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This module draws random numbers and lays out workload shapes; it
holds none of the method's arithmetic.

Generator (counter based, so any entry can be drawn independently):
    mix(z)      = SplitMix64 finaliser (Steele, Lea & Flood 2014):
                  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
                  z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    key(s, id)  = mix(s ^ mix(id + 0x632BE59BD9B4E019))
    word(s,id,i)= mix(key + (i + 1) * 0x9E3779B97F4A7C15)      (mod 2^64)
    uniform     = (word >> 11) * 2^-53  in [0, 1)
    sym_uniform = 2 * uniform - 1        in [-1, 1)
The library implements the same definition for its own seeded node
initialisation; `sym_uniform` is exact in binary64 on both sides.
Normal draws (Box-Muller on pairs of uniforms) are used only for inputs
handed over to both sides as arrays.
"""

import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
GAMMA = np.uint64(0x9E3779B97F4A7C15)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(0xBF58476D1CE4E5B9)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def words(seed, stream, n):
    with np.errstate(over="ignore"):
        key = _mix(np.uint64(seed) ^ _mix(np.uint64(stream) + np.uint64(0x632BE59BD9B4E019)))
        i = np.arange(1, n + 1, dtype=np.uint64)
        return _mix(key + i * GAMMA)


def uniform(seed, stream, n):
    return (words(seed, stream, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def sym_uniform(seed, stream, n):
    return 2.0 * uniform(seed, stream, n) - 1.0


def normal(seed, stream, n):
    m = (n + 1) // 2
    u = uniform(seed, stream, 2 * m)
    u1 = 1.0 - u[0::2]          # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def integers(seed, stream, n, lo, hi):
    """n integers uniform in [lo, hi] (inclusive), by floor of uniform."""
    u = uniform(seed, stream, n)
    return lo + np.floor(u * (hi - lo + 1)).astype(np.int64)


# ----------------------------------------------------------------------
# workload shapes (sizes and draws only)
# ----------------------------------------------------------------------
C1_LEG = [(-2, 2), (-1, 3), (0, 6), (1, 3), (2, 2)]
C4_LEG = [(-4, 4), (-3, 8), (-2, 16), (-1, 23), (0, 26), (1, 23), (2, 16), (3, 8), (4, 4)]


def symmetric_sector_op(seed, stream, leg):
    """Sector-preserving leg operator: per sector (G + G^T)/2, G ~ N(0,1).
    Returns {q: n x n array}."""
    out = {}
    tot = sum(n * n for _, n in leg)
    g = normal(seed, stream, tot)
    o = 0
    for q, n in leg:
        G = g[o:o + n * n].reshape(n, n)
        o += n * n
        out[q] = 0.5 * (G + G.T)
    return out


def single_node_terms(seed, K, leg, streams_from=100):
    """K three-factor terms, each factor a symmetric sector-preserving
    operator on the (common) leg, coefficient 1."""
    terms = []
    for k in range(K):
        ops = [symmetric_sector_op(seed, streams_from + 3 * k + j, leg) for j in range(3)]
        terms.append((1.0, ops[0], ops[1], ops[2]))
    return terms


def random_composition(seed, stream, chi, S):
    """Sizes of S sectors summing to chi: S-1 distinct cut points drawn
    uniformly from 1..chi-1 (by rejection in draw order).  S <= chi."""
    if not 1 <= S <= chi:
        raise ValueError("need 1 <= S <= chi")
    cuts = []
    draws = integers(seed, stream, 64 * S + 64, 1, max(1, chi - 1))
    i = 0
    while len(cuts) < S - 1:
        if i == len(draws):
            draws = integers(seed, stream, 2 * len(draws), 1, max(1, chi - 1))
        c = int(draws[i])
        i += 1
        if c not in cuts:
            cuts.append(c)
    cuts = sorted(cuts)
    edges = [0] + cuts + [chi]
    return [edges[a + 1] - edges[a] for a in range(S)]


def batched_leg(seed, stream, chis=(32, 48, 64, 96, 128), smin=3, smax=9):
    chi = chis[int(integers(seed, stream, 1, 0, len(chis) - 1)[0])]
    S = min(chi, int(integers(seed, stream + 1, 1, smin, smax)[0]))
    sizes = random_composition(seed, stream + 2, chi, S)
    q0 = -((S - 1) // 2)
    return [(q0 + i, sizes[i]) for i in range(S)]


def batched_nodes(seed, nnodes, chis=(32, 48, 64, 96, 128), kmin=12, kmax=24,
                  allowed=None):
    """Independent nodes of the batched workload: per leg chi ~ U(chis),
    S ~ U{3..9} sectors (charges q0 .. q0+S-1, q0 = -floor((S-1)/2)) with a
    random composition of chi; K ~ U{kmin..kmax} terms, each factor a
    symmetric sector-preserving operator, coefficient 1.  A node whose legs
    admit no block (checked by the caller-supplied `allowed(legs)`) is
    redrawn from the next stream."""
    out = []
    stream = 0
    while len(out) < nnodes:
        base = 100000 + 1000 * stream
        legs = [batched_leg(seed, base + 10 * e, chis) for e in range(3)]
        stream += 1
        if allowed is not None and not allowed(legs):
            continue
        K = int(integers(seed, base + 50, 1, kmin, kmax)[0])
        terms = []
        for k in range(K):
            ops = [symmetric_sector_op(seed, base + 100 + 3 * k + e, legs[e]) for e in range(3)]
            terms.append((1.0, ops[0], ops[1], ops[2]))
        out.append((legs, terms))
    return out


def bottom_node_pattern(lat_L):
    """Factor pattern of the effective Hamiltonian of the first bottom node
    (sites 0 and 1, the pair merged along x) of an open lattice: per term
    (hasA, dA, hasB, dB, hasC, dC), which legs carry a factor and its
    charge shift.  One block Hamiltonian per leg and class (physics,
    penalty); per link between two sides, two hopping terms (shifts +1/-1
    and -1/+1, the parent side's shift negated) and three penalty terms;
    per plaquette touching two or three sides, two terms."""
    Lx, Ly, Lz = lat_L

    def idx(i, j, k):
        return i + Lx * (j + Ly * k)

    def inside(i, j, k):
        return 0 <= i < Lx and 0 <= j < Ly and 0 <= k < Lz

    def side(s):
        return 0 if s == 0 else (1 if s == 1 else 2)

    metas = [(True, 0, False, 0, False, 0), (False, 0, True, 0, False, 0),
             (False, 0, False, 0, True, 0)] * 2
    for k in range(Lz):
        for j in range(Ly):
            for i in range(Lx):
                x = idx(i, j, k)
                for mu in range(3):
                    c = [i, j, k]
                    c[mu] += 1
                    if not inside(*c):
                        continue
                    y = idx(*c)
                    sx, sy = side(x), side(y)
                    if sx == sy:
                        continue
                    for dx, dy in ((1, -1), (-1, 1), (0, 0), (0, 0), (0, 0)):
                        has = [False] * 3
                        d = [0, 0, 0]
                        has[sx], d[sx] = True, dx if sx < 2 else -dx
                        has[sy], d[sy] = True, dy if sy < 2 else -dy
                        metas.append((has[0], d[0], has[1], d[1], has[2], d[2]))
                for a, b in ((0, 1), (0, 2), (1, 2)):
                    c1 = [i, j, k]; c1[a] += 1
                    c2 = [i, j, k]; c2[b] += 1
                    c3 = list(c1); c3[b] += 1
                    if not (inside(*c1) and inside(*c2) and inside(*c3)):
                        continue
                    sides = {side(x), side(idx(*c1)), side(idx(*c2)), side(idx(*c3))}
                    if len(sides) < 2:
                        continue
                    for _ in range(2):
                        metas.append((0 in sides, 0, 1 in sides, 0, 2 in sides, 0))
    return metas


def pattern_op_blocks(seed, legs, metas):
    """Random dense blocks for every factor of a pattern: per term and leg
    with a factor, {q: (n_{q+d} x n_q) N(0,1) block} for every input sector
    q whose shifted charge q + d is a sector (None for identities)."""
    out = []
    for t, (hA, dA, hB, dB, hC, dC) in enumerate(metas):
        ops = []
        for e, (h, d) in enumerate(((hA, dA), (hB, dB), (hC, dC))):
            if not h:
                ops.append(None)
                continue
            blk = {}
            sizes = dict(legs[e])
            for q, n in legs[e]:
                if q + d in sizes:
                    blk[q] = normal(seed, 1000 * t + 10 * e + q + 5, sizes[q + d] * n).reshape(sizes[q + d], n)
            ops.append(blk)
        out.append(ops)
    return out
