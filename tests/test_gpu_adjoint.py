"""GPU parity of the hand-written adjoint of the effective-Hamiltonian
application and of the autograd wrapper: cotangents of the node tensor,
of every factor and of every coefficient against the oracle's reverse
mode; energy derivatives against central differences of converged FP64
eigensolves and against Hellmann-Feynman expectation values."""

import numpy as np
import pytest

from oracle import blocks as oblocks
from oracle import heff as oheff
from paper_2011_10658_amd import lib, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = lib.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def flat_op(blk, leg):
    """{q_in: block} -> leg-operator layout (ascending input charge)."""
    parts = [blk[q].reshape(-1) for q, _ in leg if q in blk]
    return np.concatenate(parts) if parts else np.zeros(0)


LEG42 = [(-2, 5), (-1, 9), (0, 14), (1, 9), (2, 5)]
SHIFTS = [(1, 0, 1), (0, 0, 0), (None, -1, -1), (0, None, None), (-1, 1, None),
          (None, None, None), (0, None, 0), (2, -1, 1)]


def shifted_case(seed, leg):
    """Non-symmetric factors N(0,1) with charge shifts (identities
    included); x, ybar N(0,1) on the allowed blocks."""
    sizes = dict(leg)
    terms, dterms, metas = [], [], []
    stream = 0
    for k, sh in enumerate(SHIFTS):
        c = 1.0 - 0.25 * k
        ops, dense = [], []
        for e, d in enumerate(sh):
            if d is None:
                ops.append(None)
                dense.append(None)
                continue
            blk = {}
            for q, n in leg:
                if q + d in sizes:
                    blk[q] = synth.normal(seed, 1000 + stream, sizes[q + d] * n).reshape(sizes[q + d], n)
                    stream += 1
            ops.append(blk)
            dense.append(oblocks.op_to_dense(blk, leg, d))
        terms.append((c, ops, tuple(0 if d is None else d for d in sh)))
        dterms.append((c, *dense))
        metas.append(sh)
    legs = (leg, leg, leg)
    size = oblocks.block_table(*legs)[1][-1]
    x = synth.normal(seed, 1, size)
    yb = synth.normal(seed, 2, size)
    return legs, terms, dterms, x, yb


def upload_terms(ctx, legs, terms):
    keep, spec = [], []
    for c, ops, sh in terms:
        ptrs = []
        for e, o in enumerate(ops):
            if o is None:
                ptrs.append(0)
                continue
            t = dev(flat_op(o, legs[e]))
            keep.append(t)
            ptrs.append(t.data_ptr() if t.numel() else 0)
        spec.append((c, tuple(ptrs), sh))
    return spec, keep


def run_adjoint(ctx, legs, terms, x, yb):
    spec, keep = upload_terms(ctx, legs, terms)
    h = ctx.heff(*legs, spec)
    xd, ybd = dev(x), dev(yb)
    xbar = torch.full_like(xd, np.nan)
    opbar = []
    for c, ops, sh in terms:
        for e, o in enumerate(ops):
            n = 0 if o is None else flat_op(o, legs[e]).size
            opbar.append(torch.full((max(n, 1),), np.nan, dtype=torch.float64, device="cuda"))
    ptrs = [g.data_ptr() for g in opbar]
    cbar = h.adjoint(xd.data_ptr(), ybd.data_ptr(), xbar.data_ptr(), ptrs, True, len(terms))
    out = (xbar.cpu().numpy(), [g.cpu().numpy() for g in opbar], cbar)
    h.close()
    return out


@pytest.mark.parametrize("dtype,tol", [(lib.FP64, 1e-12), (lib.FP32, 2e-5)])
def test_adjoint_matches_oracle_shifted(ctx, dtype, tol):
    ctx.set_precision(dtype)
    legs, terms, dterms, x, yb = shifted_case(7, LEG42)
    xbar, opbar, cbar = run_adjoint(ctx, legs, terms, x, yb)
    xb_o, g_o, c_o = oheff.adjoint_dense(oblocks.to_dense(x, *legs), oblocks.to_dense(yb, *legs), dterms)
    xb_o = oblocks.from_dense(xb_o, *legs)
    assert np.abs(xbar - xb_o).max() <= tol * np.abs(xb_o).max()
    for k, (c, ops, sh) in enumerate(terms):
        for e in range(3):
            if ops[e] is None:
                assert g_o[k][e] is None
                continue
            ref = flat_op(oblocks.op_from_dense(g_o[k][e], legs[e], sh[e]), legs[e])
            got = opbar[3 * k + e][:ref.size]
            assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (k, e)
    assert np.abs(cbar - c_o).max() <= tol * np.abs(c_o).max()
    ctx.set_precision(lib.FP64)


def test_adjoint_is_deterministic_and_repeatable(ctx):
    ctx.set_precision(lib.FP32)
    legs, terms, dterms, x, yb = shifted_case(8, LEG42)
    a = run_adjoint(ctx, legs, terms, x, yb)
    b = run_adjoint(ctx, legs, terms, x, yb)
    assert np.array_equal(a[0], b[0])
    # entries for identity factors are never written (left NaN)
    assert all(np.array_equal(p, q, equal_nan=True) for p, q in zip(a[1], b[1]))
    assert np.array_equal(a[2], b[2])
    ctx.set_precision(lib.FP64)


# ----------------------------------------------------------------------
# full size: chi = 128, charges -4..4, K = 24, FP32 GEMMs
# ----------------------------------------------------------------------
C4 = synth.C4_LEG
K4 = 24
N_EL = 8          # terms 0..7 carry the electric coupling g^2 / 2


def c4_terms():
    return synth.single_node_terms(4, K4, C4)


def c4_ops(terms):
    return [dev(flat_op(o, C4)) for _, *ops in terms for o in ops]


def coefs_for(g2):
    return np.array([g2 / 2.0] * N_EL + [1.0] * (K4 - N_EL))


def heff_for(ctx, ops, coefs, dtype):
    ctx.set_precision(dtype)
    spec = [(float(coefs[k]), tuple(ops[3 * k + e].data_ptr() for e in range(3)), (0, 0, 0))
            for k in range(K4)]
    h = ctx.heff(C4, C4, C4, spec)
    ctx.set_precision(lib.FP64)
    return h


def ground(ctx, ops, coefs, x0):
    """Converged FP64 lowest eigenpair (restarted Lanczos)."""
    h = heff_for(ctx, ops, coefs, lib.FP64)
    ctx.set_lanczos(64, 400, 1e-11)
    xd = dev(x0)
    ev, res, rc = h.lanczos(xd.data_ptr(), 64)
    h.close()
    ctx.set_lanczos(30, 1, 0.0)
    assert rc == 0 and res <= 1e-11 * abs(ev)
    return ev, xd


def test_c4_adjoint_sampled_against_oracle(ctx):
    terms = c4_terms()
    ops = c4_ops(terms)
    size = oblocks.block_table(C4, C4, C4)[1][-1]
    assert size == 253604
    x, yb = synth.normal(4, 1, size), synth.normal(4, 2, size)
    coefs = coefs_for(1.0)
    h = heff_for(ctx, ops, coefs, lib.FP32)
    xd, ybd = dev(x), dev(yb)
    xbar = torch.full_like(xd, np.nan)
    sample = (0, 9, 23)
    opbar = [torch.full_like(ops[i], np.nan) if i // 3 in sample else None for i in range(3 * K4)]
    cbar = h.adjoint(xd.data_ptr(), ybd.data_ptr(), xbar.data_ptr(),
                     [0 if g is None else g.data_ptr() for g in opbar], True, K4)
    # the transposed schedule of sector-preserving square factors costs what
    # the forward one costs; every factor gradient adds work
    f_fwd, _ = h.flops()
    f_xb, f_gr = h.adjoint_flops()
    assert f_xb == f_fwd and f_gr > f_fwd
    h.close()
    legs = (C4, C4, C4)
    dterms = [(coefs[k], *(oblocks.op_to_dense(o, C4, 0) for o in t[1:])) for k, t in enumerate(terms)]
    # every factor is symmetric, so the transposed application is H itself
    xb_o = oheff.apply_flat(yb, legs, dterms)
    xbar = xbar.cpu().numpy()
    assert np.abs(xbar - xb_o).max() <= 2e-5 * np.abs(xb_o).max()
    xd_, ybd_ = oblocks.to_dense(x, *legs), oblocks.to_dense(yb, *legs)
    for k in sample:
        _, g_o, c_o = oheff.adjoint_dense(xd_, ybd_, [dterms[k]])
        for e in range(3):
            ref = flat_op(oblocks.op_from_dense(g_o[0][e], C4, 0), C4)
            got = opbar[3 * k + e].cpu().numpy()
            assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max(), (k, e)
        assert abs(cbar[k] - c_o[0]) <= 2e-5 * abs(c_o[0]) + 1e-6 * np.abs(cbar).max()


def test_c4_energy_derivative_in_g2(ctx):
    """dE0/d(g^2): autograd through the FP32 adjoint at the FP64 ground
    state, Hellmann-Feynman (1/2) sum_{k electric} <v|H_k|v> from the
    oracle, and central differences (h = 1e-4) of converged FP64
    eigenvalues all agree."""
    from paper_2011_10658_amd.autograd import HeffSpec, heff_apply

    terms = c4_terms()
    ops = c4_ops(terms)
    size = oblocks.block_table(C4, C4, C4)[1][-1]
    x0 = synth.normal(4, 3, size)
    g2 = 1.0
    E0, v = ground(ctx, ops, coefs_for(g2), x0)
    h = 1e-4
    Ep, _ = ground(ctx, ops, coefs_for(g2 + h), v.cpu().numpy())
    Em, _ = ground(ctx, ops, coefs_for(g2 - h), v.cpu().numpy())
    fd = (Ep - Em) / (2 * h)
    vn = v.cpu().numpy()
    el = [(1.0, *(oblocks.op_to_dense(o, C4, 0) for o in t[1:])) for t in terms[:N_EL]]
    hf = 0.5 * float(vn @ oheff.apply_flat(vn, (C4, C4, C4), el))
    assert abs(fd - hf) <= 1e-6 * max(1.0, abs(hf)), (fd, hf)
    # autograd, FP32 GEMMs
    ctx.set_precision(lib.FP32)
    spec = HeffSpec(ctx, (C4, C4, C4), tuple((0, 0, 0) for _ in range(K4)))
    g = torch.tensor(g2, dtype=torch.float64, requires_grad=True)
    coefs = torch.cat([(g / 2).expand(N_EL), torch.ones(K4 - N_EL, dtype=torch.float64)])
    E = torch.dot(v, heff_apply(v, coefs.cuda(), spec, ops))
    E.backward()
    ctx.set_precision(lib.FP64)
    assert abs(E.item() - E0) <= 1e-5 * abs(E0)
    assert abs(g.grad.item() - hf) <= 1e-5 * max(1.0, abs(hf)), (g.grad.item(), hf)


def test_c4_energy_derivative_in_node_tensor(ctx):
    """dE/dT for the Rayleigh quotient E(T) = <T|H|T>/<T|T> at a random T:
    autograd through the FP32 adjoint against FP64 central differences
    along random directions; at the ground state the gradient vanishes to
    the eigensolver's residual."""
    from paper_2011_10658_amd.autograd import HeffSpec, heff_apply

    terms = c4_terms()
    ops = c4_ops(terms)
    size = oblocks.block_table(C4, C4, C4)[1][-1]
    coefs = coefs_for(1.0)
    T0 = synth.normal(4, 5, size)
    h64 = heff_for(ctx, ops, coefs, lib.FP64)

    def rq(t):
        td = dev(t)
        y = torch.empty_like(td)
        h64.matvec(td.data_ptr(), y.data_ptr())
        return float(torch.dot(td, y) / torch.dot(td, td))

    ctx.set_precision(lib.FP32)
    spec = HeffSpec(ctx, (C4, C4, C4), tuple((0, 0, 0) for _ in range(K4)))
    T = dev(T0).requires_grad_(True)
    E = torch.dot(T, heff_apply(T, dev(coefs), spec, ops)) / torch.dot(T, T)
    E.backward()
    ctx.set_precision(lib.FP64)
    grad = T.grad.cpu().numpy()
    gn = np.linalg.norm(grad)
    for s in range(3):
        D = synth.normal(4, 10 + s, size)
        hstep = 1e-4
        fd = (rq(T0 + hstep * D) - rq(T0 - hstep * D)) / (2 * hstep)
        assert abs(fd - grad @ D) <= 1e-5 * gn * np.linalg.norm(D), (s, fd, grad @ D)
    h64.close()
    # at the ground state
    E0, v = ground(ctx, ops, coefs, T0)
    ctx.set_precision(lib.FP32)
    V = v.clone().requires_grad_(True)
    E = torch.dot(V, heff_apply(V, dev(coefs), spec, ops)) / torch.dot(V, V)
    E.backward()
    ctx.set_precision(lib.FP64)
    assert V.grad.norm().item() <= 1e-4 * abs(E0)


def test_c4_energy_derivative_in_an_operator(ctx):
    """dE0/dC_k along a random symmetric direction: autograd (adjoint with
    x = ybar = v) against central differences of converged FP64
    eigenvalues."""
    from paper_2011_10658_amd.autograd import HeffSpec, heff_apply

    terms = c4_terms()
    ops = c4_ops(terms)
    size = oblocks.block_table(C4, C4, C4)[1][-1]
    coefs = coefs_for(1.0)
    E0, v = ground(ctx, ops, coefs, synth.normal(4, 3, size))
    k, e = 11, 2
    Dblk = synth.symmetric_sector_op(4, 999, C4)
    D = dev(flat_op(Dblk, C4))
    hstep = 1e-4
    moved = list(ops)
    moved[3 * k + e] = ops[3 * k + e] + hstep * D
    Ep, _ = ground(ctx, moved, coefs, v.cpu().numpy())
    moved[3 * k + e] = ops[3 * k + e] - hstep * D
    Em, _ = ground(ctx, moved, coefs, v.cpu().numpy())
    fd = (Ep - Em) / (2 * hstep)
    ctx.set_precision(lib.FP32)
    spec = HeffSpec(ctx, (C4, C4, C4), tuple((0, 0, 0) for _ in range(K4)))
    leaf = [o.clone().requires_grad_(i == 3 * k + e) for i, o in enumerate(ops)]
    E = torch.dot(v, heff_apply(v, dev(coefs), spec, leaf))
    E.backward()
    ctx.set_precision(lib.FP64)
    ad = float(torch.dot(leaf[3 * k + e].grad, D))
    assert abs(ad - fd) <= 1e-5 * max(1.0, abs(fd)), (ad, fd)
    assert all(o.grad is None for i, o in enumerate(leaf) if i != 3 * k + e)
