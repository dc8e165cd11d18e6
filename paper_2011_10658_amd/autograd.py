"""torch.autograd.Function around the node-level effective Hamiltonian.

    y = HeffFunction.apply(x, coefs, spec, *ops)

applies H_eff = sum_k coefs[k] A_k (x) B_k (x) C_k to the flat block vector
x (Methods, "Tensor Networks", step (i)); backward calls the library's
hand-written adjoint, which gives the cotangents of x, of every factor and
of every coefficient.  Every step runs in libqedttn's kernels; torch only
holds the buffers and orders the stream.

Checkpointing: the forward keeps the inputs (x and the library's copy of
the factors) and nothing else; the mode-product intermediates the
gradients need are recomputed by the adjoint.  The memory held between
forward and backward is therefore |x| plus the factors, independent of the
number of terms times |x| that storing the per-term partial products would
cost.

spec = HeffSpec(qctx, legs, shifts): the library context, the three legs
[(charge, size), ...] and per term the charge shifts (dA, dB, dC).  ops
holds 3K entries: a 1-D FP64 CUDA tensor in the leg-operator layout (per
input sector in ascending charge, the n_out x n_in block row-major) or
None for the identity.  coefs is a 1-D FP64 tensor of K coefficients.
"""

from dataclasses import dataclass

import numpy as np
import torch

from . import lib


@dataclass(frozen=True)
class HeffSpec:
    qctx: "lib.Context"
    legs: tuple
    shifts: tuple


class HeffFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, coefs, spec, *ops):
        K = len(spec.shifts)
        if len(ops) != 3 * K or coefs.numel() != K:
            raise ValueError("need 3K operators and K coefficients")
        if not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("x must be a contiguous FP64 CUDA tensor")
        spec.qctx.set_stream(torch.cuda.current_stream(x.device).cuda_stream)
        cs = coefs.detach().double().cpu().tolist()
        terms = []
        for k in range(K):
            ptrs = []
            for e in range(3):
                o = ops[3 * k + e]
                if o is not None and (not o.is_cuda or o.dtype != torch.float64 or not o.is_contiguous()):
                    raise ValueError("operators must be contiguous FP64 CUDA tensors")
                ptrs.append(0 if o is None else o.data_ptr())
            terms.append((cs[k], tuple(ptrs), tuple(spec.shifts[k])))
        h = spec.qctx.heff(*spec.legs, terms)
        if h.size != x.numel():
            h.close()
            raise ValueError(f"x has {x.numel()} entries, the node has {h.size}")
        y = torch.empty_like(x)
        h.matvec(x.data_ptr(), y.data_ptr())
        ctx.h = h
        ctx.K = K
        ctx.coef_meta = (coefs.dtype, coefs.device)
        ctx.op_meta = [None if o is None else (o.shape, o.device) for o in ops]
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, ybar):
        (x,) = ctx.saved_tensors
        h = ctx.h
        ybar = ybar.contiguous().double()
        need_x = ctx.needs_input_grad[0]
        need_c = ctx.needs_input_grad[1]
        xbar = torch.empty_like(x) if need_x else None
        opbar, ptrs = [], []
        for i, m in enumerate(ctx.op_meta):
            if m is not None and ctx.needs_input_grad[3 + i]:
                g = torch.zeros(m[0], dtype=torch.float64, device=m[1])
                opbar.append(g)
                ptrs.append(g.data_ptr())
            else:
                opbar.append(None)
                ptrs.append(0)
        cb = h.adjoint(x.data_ptr(), ybar.data_ptr(), xbar.data_ptr() if need_x else 0,
                       ptrs if any(ptrs) else None, want_coefbar=need_c, K=ctx.K)
        cbar = None
        if need_c:
            cbar = torch.from_numpy(np.asarray(cb)).to(dtype=ctx.coef_meta[0], device=ctx.coef_meta[1])
        h.close()
        ctx.h = None
        return (xbar, cbar, None, *opbar)


def heff_apply(x, coefs, spec, ops):
    """Differentiable y = H_eff x (see HeffFunction)."""
    return HeffFunction.apply(x, coefs, spec, *ops)
