"""torch.autograd wrappers of the BSE entry points.

Each function takes a Plan that was built from the W_R / eps tensors passed
alongside it; those tensors are the differentiable inputs.  Gradients follow
PyTorch's convention dL = Re sum conj(g) d(theta), which is also the C ABI's:

* apply:   Y = A(W_R, eps) X;  g_X = A g_Y (A is Hermitian), g_W_R and g_eps from
           bse_apply_adjoint with Ybar = g_Y;
* lowest_exciton_energy:  Omega_1 by block LOBPCG; Hellmann-Feynman
           dOmega_1 = x^H dA x, i.e. the adjoint with Ybar = X = x;
* haydock_spectrum: S[b][w] from the Haydock chains; backward through the
           Krylov resolvent of the stored Lanczos basis (bse_haydock_vjp).
"""
import numpy as np
import torch

from . import bse as _b


class _Apply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, W_R, eps, plan):
        ctx.plan = plan
        ctx.save_for_backward(X)
        return plan.apply(X.contiguous())

    @staticmethod
    def backward(ctx, gY):
        (X,) = ctx.saved_tensors
        plan = ctx.plan
        gY = gY.contiguous()
        gX = plan.apply(gY) if ctx.needs_input_grad[0] else None
        need_w, need_e = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gW = ge = None
        if need_w or need_e:
            g = plan.apply_adjoint(gY, X, want_WR=need_w, want_eps=need_e)
            gW, ge = g["W_R"], g["eps"]
        return gX, gW, ge, None


def apply(plan, X, W_R, eps):
    """Y = A X, differentiable in X, W_R ([n_R][n_aux][n_aux]) and eps ([Nk][nv+nc])."""
    return _Apply.apply(X, W_R, eps, plan)


class _Lowest(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W_R, eps, plan, n_block, tol, max_iter):
        omega, x, _ = plan.lowest_excitons(n_block=n_block, max_iter=max_iter, tol=tol)
        ctx.plan = plan
        ctx.save_for_backward(x[:, :1].contiguous())
        return torch.tensor(omega[0], dtype=torch.float64, device=W_R.device)

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        need_w, need_e = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        out = ctx.plan.apply_adjoint(x, x, want_WR=need_w, want_eps=need_e)
        s = g.to(torch.float64)
        gW = out["W_R"] * s if need_w else None
        ge = out["eps"] * s if need_e else None
        return gW, ge, None, None, None, None


# LOBPCG residual tolerance per plan precision: the residual of an FP32 or BF16x3 operator cannot fall
# below its rounding (about 4e-8 of |A| for BF16x3), so those plans converge to 1e-6
LOBPCG_TOL = {"f64": 1e-10, "f32": 1e-6, "bf16x3": 1e-6}


def lowest_exciton_energy(plan, W_R, eps, n_block=4, tol=None, max_iter=300):
    """Omega_1 (the lowest TDA eigenvalue) with its Hellmann-Feynman gradient; tol defaults to the
    residual the plan's precision can reach."""
    if tol is None:
        tol = LOBPCG_TOL[plan.prec]
    return _Lowest.apply(W_R, eps, plan, n_block, tol, max_iter)


class _Spectrum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W_R, eps, plan, P, n_steps, omega, eta):
        out = plan.haydock(P, n_steps, omega, eta, keep_basis=True)
        ctx.plan, ctx.out, ctx.omega, ctx.eta = plan, out, np.asarray(omega, dtype=np.float64), eta
        return torch.as_tensor(out["S"], dtype=torch.float64, device=W_R.device)

    @staticmethod
    def backward(ctx, gS):
        need_w, need_e = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gamma = gS.detach().to("cpu", torch.float64).numpy()
        g = ctx.plan.haydock_vjp(ctx.out, ctx.omega, ctx.eta, gamma, want_WR=need_w, want_eps=need_e)
        return g["W_R"], g["eps"], None, None, None, None, None


def haydock_spectrum(plan, P, W_R, eps, n_steps, omega, eta):
    """S[b][w] of the Haydock chains started from the columns of P, differentiable in W_R and eps."""
    return _Spectrum.apply(W_R, eps, plan, P, n_steps, omega, eta)
