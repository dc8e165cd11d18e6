"""The allocation-free H_eff matvec (stage workspace in the library's
fixed per-GPU scratch) against the ordinary matvec through the C ABI:
two calls in a row on the same GPU, the second on a smaller node, each
equal to qed_heff_matvec on the same input (same plan and kernels, so the
results agree bit for bit, which is stricter than the oracle tolerances
those calls are held to); a node whose workspace exceeds the scratch is
refused before anything runs."""

import numpy as np
import pytest

from paper_2011_10658_amd import lib, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def node(ctx, leg, K, seed):
    keep, spec = [], []
    for c, a, b, cc in synth.single_node_terms(seed, K, leg):
        ptrs = []
        for o in (a, b, cc):
            t = dev(np.concatenate([o[q].reshape(-1) for q, _ in leg]))
            keep.append(t)
            ptrs.append(t.data_ptr())
        spec.append((c, tuple(ptrs), (0, 0, 0)))
    return ctx.heff(leg, leg, leg, spec), keep


@pytest.mark.parametrize("dtype", [lib.FP64, lib.FP32])
def test_noalloc_matvec_equals_matvec(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = lib.Context(0)
    ctx.set_precision(dtype)
    try:
        # first a larger node (legs 128^3, 9 sectors, 253,604 entries,
        # 6 terms), then the smaller single-node workload (792 entries)
        for leg, K, seed in ((synth.C4_LEG, 6, 4), (synth.C1_LEG, 8, 1)):
            h, keep = node(ctx, leg, K, seed)
            x = dev(synth.normal(seed, 11, h.size))
            y_ref = torch.full((h.size,), np.nan, dtype=torch.float64, device="cuda")
            y_na = torch.full((h.size,), np.nan, dtype=torch.float64, device="cuda")
            h.matvec(x.data_ptr(), y_ref.data_ptr())
            h.matvec_noalloc(x.data_ptr(), y_na.data_ptr())
            torch.cuda.synchronize()
            a, b = y_ref.cpu().numpy(), y_na.cpu().numpy()
            assert np.isfinite(a).all()
            assert np.array_equal(a, b), np.abs(a - b).max()
            h.close()
    finally:
        ctx.close()


def test_noalloc_rejects_oversized_workspace():
    """A node whose stage intermediates exceed the scratch: the call fails
    with an error before any kernel runs; the ordinary matvec still works."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = lib.Context(0)
    ctx.set_precision(lib.FP64)
    try:
        leg = synth.C4_LEG
        h, keep = node(ctx, leg, 48, 5)
        x = dev(synth.normal(5, 11, h.size))
        y = torch.zeros(h.size, dtype=torch.float64, device="cuda")
        with pytest.raises(lib.QedError) as ei:
            h.matvec_noalloc(x.data_ptr(), y.data_ptr())
        assert ei.value.code == -1   # QED_ERR_INVALID_ARG
        assert "workspace" in str(ei.value)
        h.matvec(x.data_ptr(), y.data_ptr())
        torch.cuda.synchronize()
        assert np.isfinite(y.cpu().numpy()).all()
        h.close()
    finally:
        ctx.close()
