"""torch.autograd.Function over the cooling step (differentiation form).

``CoolStep.apply(tables, n_e, T_e, T_i, B, H, table_param, dt, opts)`` returns
(T_e_new, T_i_new, Q_rad, Q_cc).  The backward pass is the library's adjoint
kernel (rc_cool_step_backward): gradients flow to the five state tensors and,
through ``table_param`` (a float64 tensor of n_values entries standing for the
log2 table node values, e.g. ``torch.zeros(n_values, requires_grad=True)``),
to every table entry.  The table values themselves are those held by
``tables``; ``table_param`` only carries their gradient.
"""
import torch

from . import radcool


class CoolStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tables, n_e, T_e, T_i, B, H, table_param, dt, opts=None):
        opts = opts or radcool.default_opts()
        state = {"n_e": n_e.detach(), "T_e": T_e.detach(), "T_i": T_i.detach(), "B": B.detach(), "H": H.detach()}
        out = radcool.cool_step(tables, state, dt, opts)
        ctx.tables = tables
        ctx.dt = dt
        ctx.opts = opts
        ctx.save_for_backward(n_e, T_e, T_i, B, H, out["T_e_new"], out["T_i_new"], out["status"])
        ctx.mark_non_differentiable(out["status"])
        return out["T_e_new"], out["T_i_new"], out["Q_rad"], out["Q_cc"], out["status"]

    @staticmethod
    def backward(ctx, g_te, g_ti, g_qr, g_qc, _g_status):
        n_e, T_e, T_i, B, H, te_new, ti_new, status = ctx.saved_tensors
        state = {"n_e": n_e, "T_e": T_e, "T_i": T_i, "B": B, "H": H}
        fwd = {"T_e_new": te_new, "T_i_new": ti_new, "status": status}
        cot = {"T_e_new": g_te, "T_i_new": g_ti, "Q_rad": g_qr, "Q_cc": g_qc}
        tg = None
        if ctx.needs_input_grad[6]:
            _, nv = ctx.tables.info()
            tg = torch.zeros(nv, dtype=torch.float64, device=n_e.device)
        g = radcool.cool_step_backward(ctx.tables, state, ctx.dt, fwd, cot, ctx.opts, table_grad=tg)
        return None, g["n_e"], g["T_e"], g["T_i"], g["B"], g["H"], tg, None, None


def radiated_energy(n_e, T_e, T_i, T_e_new, T_i_new):
    """Total radiated energy per unit volume, sum over cells of
    1.5 n_e k (T_e + T_i - T_e' - T_i') (u = n k T / (gamma - 1), gamma = 5/3)."""
    k_B = 1.380649e-16
    return (1.5 * n_e * k_B * ((T_e + T_i) - (T_e_new + T_i_new))).sum()
