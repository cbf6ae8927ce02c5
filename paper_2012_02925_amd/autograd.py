"""torch.autograd bindings of the hand-written adjoint.

ResidualFn          R(Q) as a differentiable op: forward cfd_residual,
                    backward cfd_residual_vjp (the solver's own state is put
                    back after each pass).
UnrolledWallPressure J(theta, X) = integrated wall pressure after n Runge-Kutta
                    steps from the uniform state theta (inflow state, also the
                    inflow boundary value) on nodes X.  Forward keeps a
                    checkpoint (bit-exact copy of the solution) every `every`
                    steps and records the stage states of the last segment as
                    it computes them; backward reverses that segment at once,
                    then replays each earlier segment from its checkpoint with
                    cfd_rk_step_record (ghost-filled stage states of every step
                    of the segment) and reverses it with
                    cfd_rk_step_vjp_recorded.

All arithmetic runs in the library's kernels; this module only sequences the
calls and marshals tensors.
"""
import torch


class ResidualFn(torch.autograd.Function):
    """R(Q) at the state Q (packed conservative, (nvar, ncells)).  Both passes
    evaluate at Q through the solver's context and then put back the state
    the solver held before (bit-exact copy), so calling this op does not
    disturb a run in progress."""

    @staticmethod
    def forward(ctx, Q, solver):
        with _state_kept(solver):
            solver.set_state(Q)
            R = solver.residual()
        ctx.solver = solver
        ctx.save_for_backward(Q)
        return R

    @staticmethod
    def backward(ctx, Rbar):
        (Q,) = ctx.saved_tensors
        s = ctx.solver
        with _state_kept(s):
            s.set_state(Q)
            Qbar, _, _ = s.residual_vjp(Rbar.contiguous())
        return Qbar, None


class _state_kept:
    """Save the solver's current state (if it holds one) and restore it on exit."""

    def __init__(self, solver):
        self.s = solver
        self.buf = None

    def __enter__(self):
        if self.s.has_state:
            self.buf = self.s.save_state()
        return self

    def __exit__(self, *exc):
        if self.buf is not None:
            self.s.load_state(self.buf)
        return False


def residual(solver, Q):
    return ResidualFn.apply(Q, solver)


def _uniform_prims(solver, theta):
    th = theta.detach().to(device=solver.device, dtype=torch.float64)
    return th.reshape(-1, 1).expand(solver.nvar, solver.ncells).contiguous()


class UnrolledWallPressure(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, nodes, solver, nsteps, every, inflow_patch):
        s = solver
        s.inflow_slot(inflow_patch)  # rejects a patch that is not a supersonic inflow
        s.set_nodes(nodes.detach())
        th = [float(x) for x in theta.detach().cpu()]
        s.set_bc_params(inflow_patch, th)
        s.set_state_primitive(_uniform_prims(s, theta))
        ckpts = []
        last = ((nsteps - 1) // every) * every if nsteps > 0 else 0
        slots, per = s.stage_record_buffer(every)
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append((n, s.save_state()))
            if n >= last:
                s.rk_step_record(slots[(n - last) * per:(n - last + 1) * per])
            else:
                s.rk_step(1)
        J, _ = s.objective_wall_pressure(with_grad=False)
        if not any(ctx.needs_input_grad[:2]):  # no backward will follow
            s.release_record_buffer(slots)
            slots = None
        ctx.solver, ctx.nsteps, ctx.every, ctx.th = s, nsteps, every, th
        ctx.slot = s.inflow_slot(inflow_patch)
        ctx.ckpts = ckpts
        ctx.slots, ctx.per, ctx.last = slots, per, last
        ctx.final = s.save_state()
        ctx.theta_device = theta.device
        ctx.nodes_shape = nodes.shape
        return J.reshape(()).to(theta.device)

    @staticmethod
    def backward(ctx, Jbar):
        s = ctx.solver
        s.adjoint_reset()
        s.load_state(ctx.final)
        _, Qbar = s.objective_wall_pressure(with_grad=True)
        Qbar = Qbar.contiguous()
        slots, per = ctx.slots, ctx.per
        for (start, buf) in reversed(ctx.ckpts):
            end = min(start + ctx.every, ctx.nsteps)
            if start != ctx.last:  # the last segment was recorded by the forward pass
                s.load_state(buf)
                for n in range(end - start):
                    s.rk_step_record(slots[n * per:(n + 1) * per])
            for n in reversed(range(end - start)):
                s.rk_step_vjp_recorded(slots[n * per:(n + 1) * per], Qbar)
        s.release_record_buffer(slots)
        ctx.slots = None
        Xbar, Tbar = s.adjoint_result(nodes=True, inflow=True)
        theta_bar = s.uniform_state_vjp(ctx.th, Qbar) + Tbar[ctx.slot]
        jb = Jbar.to(s.device)
        return (jb * theta_bar).to(ctx.theta_device), (jb * Xbar).reshape(ctx.nodes_shape), None, None, None, None


def unrolled_wall_pressure(solver, theta, nodes, nsteps, every=10, inflow_patch=0):
    return UnrolledWallPressure.apply(theta, nodes, solver, nsteps, every, inflow_patch)
