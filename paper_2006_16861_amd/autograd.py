"""Differentiable Helmholtz solve: U = H(m)^-1 F as a torch.autograd.Function.

Forward: build the operator from the squared slowness m = 1/c^2 at the nodes
(c = m^-1/2), then solve H U = F for every right-hand side with the
time-domain preconditioned GMRES of libtdp.

Backward, for a real loss L with incoming gradient g = dL/dRe U + i dL/dIm U
(torch's convention for complex tensors): dU = H^-1 (dF - dH U), so
    dL = Re<lam, dF> - Re<lam, dH U>,   lam = H^-H g.
H is complex symmetric (Re H symmetric, Im H diagonal: Sec. 1 eqs. 9-10 and
Sec. 2.2), so H^-H = conj(H)^-1 and lam = conj(H^-1 conj(g)): the adjoint is
one more solve with the same operator and preconditioner.  Then
grad_F = lam and, since dH/dm_cell = -omega^2 M_cell (App. A cell form) and
m_cell is the corner average of m,
    dL/dm_cell = omega^2 Re sum_{b,g in cell} M[Delta(b,g)] conj(lam_b) U_g,
mapped to the nodes by the adjoint of the corner averaging (tdp_grad_m).
"""
from __future__ import annotations

import torch

from . import tdp


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, F, R, omega, h, cfg):
        c = torch.rsqrt(m.detach()).contiguous()
        op = tdp.Operator(c, R, omega, h, prec=cfg.get("prec", tdp.F64),
                          steps_per_period=cfg.get("steps_per_period", 0))
        kw = dict(T=cfg["T"], rho=cfg.get("rho", 0.25), tol=cfg.get("tol", 1e-10),
                  restart=cfg.get("restart", 30), max_iters=cfg.get("max_iters", 3000),
                  variant=cfg.get("variant", 0))
        batched = F.dim() == m.dim() + 1
        Fs = F.detach() if batched else F.detach().unsqueeze(0)
        outs, infos = [], []
        for s in range(Fs.shape[0]):
            U, info = op.solve(Fs[s].contiguous(), **kw)
            if info.status != 0:
                raise RuntimeError(f"forward solve {s} did not converge: {info}")
            outs.append(U)
            infos.append(info)
        U = torch.stack(outs) if batched else outs[0]
        ctx.op, ctx.kw, ctx.batched, ctx.infos = op, kw, batched, infos
        ctx.save_for_backward(U)
        return U

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        op, kw = ctx.op, ctx.kw
        Us = U if ctx.batched else U.unsqueeze(0)
        gs = gU if ctx.batched else gU.unsqueeze(0)
        lams = []
        grad_m = None
        for s in range(Us.shape[0]):
            g = gs[s].contiguous()
            if not torch.any(g != 0):
                lam = torch.zeros_like(g)
            else:
                w, info = op.solve(torch.conj(g).resolve_conj().contiguous(), **kw)
                if info.status != 0:
                    raise RuntimeError(f"adjoint solve {s} did not converge: {info}")
                lam = torch.conj(w).resolve_conj().contiguous()
            lams.append(lam)
            gm = op.grad_m(lam, Us[s].contiguous())
            grad_m = gm if grad_m is None else grad_m + gm
        grad_F = torch.stack(lams) if ctx.batched else lams[0]
        return grad_m, grad_F, None, None, None, None


def helmholtz_solve(m, F, R, omega, h, T, **cfg):
    """U = H(m)^-1 F, differentiable in m (squared slowness at the nodes, FP64
    tensor on the GPU) and F (complex128, shape n or [S, *n]).  R: damping at
    the nodes (FP64, not differentiated).  cfg: rho, tol (default 1e-10),
    restart, max_iters, variant, prec, steps_per_period."""
    cfg = dict(cfg)
    cfg["T"] = int(T)
    return _Solve.apply(m, F, R, float(omega), float(h), cfg)
