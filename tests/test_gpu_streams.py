"""GPU: the context's stream and allocator hooks.  Sweeps from one seed
give the same energies on the default stream, after a switch to a caller's
stream made while released blocks of the default stream sit in the
context's block cache, and with device memory from a caller's allocator
(every block returned when the context closes)."""

import pytest

from paper_2011_10658_amd import lib

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def configure(ctx, dtype):
    ctx.set_lattice(2, 2, 1, lib.BC_OPEN_ZERO_FLUX)
    ctx.set_couplings(1.0, 0.7, 1.3, 0.9)
    ctx.set_charge_sector(0)
    ctx.set_bond_dim(32)
    ctx.set_penalty(20.0, 0, 0)
    ctx.set_lanczos(24, 2, 1e-13)
    ctx.set_precision(dtype)
    ctx.build_hamiltonian()
    ctx.init_state(3)


def energies(ctx, n):
    return [r["energy"] for r in ctx.sweep(n)]


@pytest.fixture(scope="module")
def reference():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = {}
    for dt in (lib.FP64, lib.FP32):
        ctx = lib.Context(0)
        configure(ctx, dt)
        out[dt] = energies(ctx, 4)
        ctx.close()
    return out


def close(a, b):
    return all(abs(x - y) <= 1e-12 * max(1.0, abs(y)) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype", [lib.FP64, lib.FP32])
def test_switch_to_user_stream(reference, dtype):
    ctx = lib.Context(0)
    configure(ctx, dtype)
    first = energies(ctx, 2)          # default stream; released blocks cached
    s = torch.cuda.Stream()           # default priority
    ctx.set_stream(s.cuda_stream)
    second = energies(ctx, 2)
    ctx.close()
    s.synchronize()
    assert close(first + second, reference[dtype]), (first + second, reference[dtype])


def test_allocator_hook(reference):
    ctx = lib.Context(0)
    held = {}

    def alloc(n, stream):
        p = torch.cuda.caching_allocator_alloc(n, 0)
        held[p] = n
        return p

    def free(p, stream):
        held.pop(p)
        torch.cuda.caching_allocator_delete(p)

    ctx.set_allocator(alloc, free)
    configure(ctx, lib.FP64)
    e = energies(ctx, 4)
    assert held                       # the library's buffers came from the hook
    ctx.close()
    torch.cuda.synchronize()
    assert not held, f"{len(held)} blocks not returned"
    assert close(e, reference[lib.FP64]), (e, reference[lib.FP64])
