"""Differentiable lAIR solve: x = A(c)^{-1} b with A(c) = A0 + diag(c).

The forward pass builds an lAIR hierarchy for A(c) and runs the stationary
V-cycle iteration; the backward pass solves the adjoint system
A(c)^T lam = dJ/dx with the transposed cycle of the same hierarchy
(pre-relaxation C, F, F on A^T, restriction with P^T, interpolation with
R^T).  Then dJ/db = lam and dJ/dc_k = -lam_k x_k, because
dA/dc_k = e_k e_k^T.  Both solves run in liblair's kernels.
"""
import torch

from . import setup as _setup


def _diag_positions(rowptr, col):
    """Index of the diagonal entry of each row (CSR on the device)."""
    n = rowptr.shape[0] - 1
    rows = torch.repeat_interleave(torch.arange(n, device=col.device),
                                   (rowptr[1:] - rowptr[:-1]).long())
    pos = torch.nonzero(col.long() == rows, as_tuple=False).squeeze(1)
    if pos.shape[0] != n:
        raise ValueError("every row needs a stored diagonal entry")
    return pos


class LairSolve(torch.autograd.Function):
    """x = LairSolve.apply(b, c, rowptr, col, val0, opts)

    b: (n,) or (n, nrhs) float64 CUDA tensor; c: (n,) float64 CUDA tensor
    added to the diagonal of the CSR matrix (rowptr, col, val0);
    opts: dict of lair.setup keyword arguments plus rtol, maxit and
    optionally reuse, a dict the caller keeps across calls: the first call
    stores its hierarchy there and later calls only replace its diagonal
    (lair_update_diag) instead of setting up again.  The shared hierarchy
    remembers whose diagonal it holds; a backward pass whose forward
    diagonal has since been replaced puts that diagonal back first (the
    same diagonal rebuilds the same hierarchy), so forward, forward,
    backward, backward gives each backward its own A(c)^T.
    """

    @staticmethod
    def forward(ctx, b, c, rowptr, col, val0, opts):
        opts = dict(opts or {})
        rtol = opts.pop("rtol", 1e-10)
        maxit = opts.pop("maxit", 200)
        reuse = opts.pop("reuse", None)
        pos = _diag_positions(rowptr, col)
        val = val0.clone()
        val[pos] += c
        diag = val[pos].contiguous()
        if reuse is not None and reuse.get("h") is not None:
            h = reuse["h"]
            h.update_diag(diag)
        else:
            h = _setup(rowptr, col, val, **opts)
            if reuse is not None:
                reuse["h"] = h
        token = None
        if reuse is not None:
            token = reuse.get("count", 0) + 1
            reuse["count"] = token
            reuse["current"] = token
        x, info = h.solve(b.contiguous(), rtol=rtol, maxit=maxit)
        if not info["converged"]:
            raise RuntimeError("lAIR forward solve did not converge: %r" % info)
        ctx.h = h
        ctx.keep = reuse is not None
        ctx.reuse, ctx.token = reuse, token
        ctx.diag = diag if reuse is not None else None
        ctx.rtol, ctx.maxit = rtol, maxit
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        if ctx.reuse is not None and ctx.reuse.get("current") != ctx.token:
            # a later forward replaced the diagonal: restore this one's
            ctx.h.update_diag(ctx.diag)
            ctx.reuse["current"] = ctx.token
        lam, info = ctx.h.solve_transpose(gx.contiguous(), rtol=ctx.rtol * 1e-2,
                                          maxit=ctx.maxit)
        if not info["converged"]:
            raise RuntimeError("lAIR adjoint solve did not converge: %r" % info)
        gb = lam if ctx.needs_input_grad[0] else None
        gc = None
        if ctx.needs_input_grad[1]:
            gc = -(lam * x) if lam.dim() == 1 else -(lam * x).sum(dim=1)
        if not ctx.keep:
            ctx.h.free()
        return gb, gc, None, None, None, None
