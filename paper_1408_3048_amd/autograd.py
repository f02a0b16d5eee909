"""Differentiable GLS map: a torch.autograd.Function over the C-ABI.

Forward: m_hat = A^-1 P^T N^-1 d for the TOD d and the per-interval noise parameters
psd = (sigma, f_knee, alpha) [Sect. 2.1, eq. glsSol].  Backward: one more PCG solve
mu = A^-1 g with g = dL/dm_hat, then dL/dd = N^-1 P mu and the noise-parameter
gradients from the lag correlations of P mu and d - P m_hat with the tap derivatives
(mm_adjoint).  No CG iterate is stored: the backward pass solves its own system.
"""

from __future__ import annotations

import numpy as np
import torch

from ._lib import Plan, _check


class GLSMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d, psd, geometry, options):
        pix, weights, n_pix, offsets = geometry
        # checked before the plan is built: the library reads d through its raw pointer
        _check(d, "d", (torch.float32, torch.float64), int(pix.shape[0]))
        opts = dict(options)
        precond = opts.pop("precond", "bj")
        precision = opts.pop("precision", "fp64")
        tol = opts.pop("tol", 1e-10)
        max_iter = opts.pop("max_iter", 3000)
        plan = Plan(pix, weights, n_pix, offsets, psd.detach().cpu().numpy().astype(np.float64),
                    precision="mixed" if precision != "fp64" else "fp64",
                    coarse=precond in ("2lvl", "adef2"), **opts)
        d_det = d.detach().contiguous()
        b = plan.rhs(d_det)
        m, _ = plan.pcg_solve(b, precond=precond, precision=precision, tol=tol,
                              max_iter=max_iter, history=False)
        ctx.plan = plan
        ctx.solve = (precond, precision, tol, max_iter)
        ctx.psd_meta = (psd.dtype, psd.device)
        ctx.save_for_backward(d_det, m)
        return m

    @staticmethod
    def backward(ctx, g):
        d, m = ctx.saved_tensors
        precond, precision, tol, max_iter = ctx.solve
        gd, gp, _, _ = ctx.plan.adjoint(m, g.detach().contiguous().to(torch.float64), d,
                                        precond=precond, precision=precision, tol=tol,
                                        max_iter=max_iter, grad_d_dtype=d.dtype)
        dtype, device = ctx.psd_meta
        return gd, torch.from_numpy(gp).to(dtype=dtype, device=device), None, None


def gls_map(d, psd, pix, weights, n_pix, offsets, **options):
    """The GLS map of TOD d (CUDA tensor) with per-interval noise parameters psd
    ([K, 3] tensor of (sigma, f_knee, alpha)), differentiable in both.  options: the
    Plan keyword arguments (n_stokes, lam, f_samp, window, fft lengths, ...) plus
    precond ("bj" / "2lvl" / "adef2"), precision ("fp64" / "mixed"), tol and max_iter of both solves."""
    return GLSMap.apply(d, psd, (pix, weights, n_pix, offsets), tuple(sorted(options.items())))
