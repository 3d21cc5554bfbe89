"""torch.autograd wrappers of the PM force and its vector-Jacobian product.

    acc = force(disp, omega_m, plan)            # a = -grad phi~ at q + disp
    disp_bar, omega_m_bar = force_vjp(disp, acc_bar, omega_m, plan)

The forward is pm_force (CIC paint, R2C, Poisson gradient, 3 C2R, CIC
readout; Sec. 2.2) and the backward is pm_force_vjp (the scatter and gather
VJPs of Sec. 3.6), so gradients through `force` are the library's own exact
discrete VJP, not automatic differentiation.  omega_m may be a Python float
or a 0-d tensor; when it is a tensor that requires grad, its gradient is
sum(acc_bar . a) / Omega_m (the force is proportional to Omega_m).

Argument marshalling only: the numbers come from libpm's kernels.
"""
import torch


def _om(omega_m):
    return float(omega_m.detach().cpu()) if isinstance(omega_m, torch.Tensor) else float(omega_m)


class Force(torch.autograd.Function):
    @staticmethod
    def forward(ctx, disp, omega_m, plan):
        om = _om(omega_m)
        acc = plan.force(disp.detach().contiguous(), om)
        ctx.save_for_backward(disp.detach())
        ctx.plan, ctx.om = plan, om
        ctx.om_is_tensor = isinstance(omega_m, torch.Tensor)
        return acc

    @staticmethod
    def backward(ctx, acc_bar):
        (disp,) = ctx.saved_tensors
        plan = ctx.plan
        xbar, ombar, _ = plan.force_vjp(disp.contiguous(), acc_bar.to(plan.mdt).contiguous(), ctx.om,
                                        want_acc=False)
        g_disp = xbar.to(disp.dtype) if ctx.needs_input_grad[0] else None
        g_om = None
        if ctx.om_is_tensor and ctx.needs_input_grad[1]:
            g_om = ombar.reshape(())
        return g_disp, g_om, None


def force(disp, omega_m, plan):
    """PM accelerations [3, N_p] (plan mesh dtype) at the lattice positions
    displaced by disp ([3, N_p], plan state dtype), differentiable in disp and
    in omega_m (when it is a tensor)."""
    return Force.apply(disp, omega_m, plan)


def force_vjp(disp, acc_bar, omega_m, plan):
    """(disp_bar, omega_m_bar) for the cotangent acc_bar of force(disp,
    omega_m): one pm_force_vjp call; omega_m_bar is a device FP64 scalar."""
    xbar, ombar, _ = plan.force_vjp(disp.contiguous(), acc_bar.to(plan.mdt).contiguous(), _om(omega_m),
                                    want_acc=False)
    return xbar, ombar.reshape(())
