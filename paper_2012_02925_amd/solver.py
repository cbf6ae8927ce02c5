"""Solver: a thin owner of one libcfdhip context.

Torch supplies the device memory (the workspace and every input/output
tensor) and the stream; all arithmetic runs in the library's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import capi
from .capi import check, dptr, int2

F64 = torch.float64


def config_from_scheme(dim, scheme, debug_flags=0):
    cfg = capi.CfdConfig()
    cfg.debug_flags = int(debug_flags)
    cfg.dim = dim
    cfg.gamma = scheme.gamma
    cfg.limiter = capi.LIM[scheme.limiter]
    cfg.muscl_eps = scheme.muscl_eps
    cfg.muscl_kappa = scheme.muscl_kappa
    le = list(scheme.lim_eps) if scheme.lim_eps is not None else [0.0] * (dim + 2)
    for v in range(5):
        cfg.lim_eps[v] = float(le[v]) if v < len(le) else 0.0
    cfg.efix = scheme.efix
    cfg.rk_stages = scheme.rk_stages
    cfg.rk_scheme = capi.RK[getattr(scheme, "rk_scheme", "mstage")]
    cfg.flux = capi.FLUX[getattr(scheme, "flux", "roe")]
    cfg.viscosity = float(getattr(scheme, "viscosity", 0.0))
    cfg.prandtl = float(getattr(scheme, "prandtl", 0.72))
    if scheme.dt_fixed is not None:
        cfg.dt_mode = capi.DT_FIXED
        cfg.dt_fixed = float(scheme.dt_fixed)
    elif getattr(scheme, "local_dt", False):
        cfg.dt_mode = capi.DT_LOCAL
        cfg.cfl = scheme.cfl
    else:
        cfg.dt_mode = capi.DT_CFL
        cfg.cfl = scheme.cfl
    return cfg


class Solver:
    """One context: blocks, boundary patches, connections and a bound workspace."""

    def __init__(self, dim, scheme, device="cuda", debug_flags=0):
        self.lib = capi.load()
        self.dim = dim
        self.nvar = dim + 2
        self.stages = scheme.rk_stages
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.cfg = config_from_scheme(dim, scheme, debug_flags)
        ctx = ctypes.c_void_p()
        check(self.lib.cfd_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(ctx)))
        self.ctx = ctx
        self.workspace = None
        self.has_state = False  # a solution has been set (set_state*, load_state)
        self._record_pool = []
        self.block_shapes = []
        self.patch_ids = []
        self.patch_kinds = []

    # -- construction ------------------------------------------------------
    @classmethod
    def from_case(cls, case, device="cuda", state=True, adjoint=False, freezing=False, debug_flags=0):
        s = cls(case.dim, case.scheme, device, debug_flags)
        if adjoint:
            s.enable_adjoint()
        if freezing:
            s.enable_limiter_freezing()
        for b in case.blocks:
            s.add_block(b.ni, b.nj, b.nk, b.nodes)
        for p in case.bcs:
            s.patch_ids.append(s.set_bc(p.block, p.face, p.lo, p.hi, p.kind, p.params))
            s.patch_kinds.append(p.kind)
        for c in case.conns:
            s.connect(c.block_a, c.face_a, c.lo_a, c.hi_a, c.block_b, c.face_b, c.lo_b, c.hi_b, c.orient)
        s.finalize_and_bind()
        if state:
            s.set_state_primitive(s.pack(case.prims))
        return s

    def _check(self, status):
        return check(status, self.ctx)

    def add_block(self, ni, nj, nk, nodes):
        arr = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
        bid = ctypes.c_int()
        self._check(self.lib.cfd_add_block(self.ctx, ni, nj, nk, arr.ctypes.data_as(capi._DP), ctypes.byref(bid)))
        self.block_shapes.append((ni, nj, nk))
        return bid.value

    def set_bc(self, block, face, lo, hi, kind, params=None):
        pid = ctypes.c_int(-1)
        par = None
        if params is not None:
            arr = (ctypes.c_double * 5)(*([float(x) for x in params] + [0.0] * (5 - len(params))))
            par = ctypes.cast(arr, capi._DP)
        self._check(self.lib.cfd_set_bc(self.ctx, block, face, int2(lo), int2(hi), capi.BC[kind], par,
                                        ctypes.byref(pid)))
        return pid.value

    def connect(self, a, fa, loa, hia, b, fb, lob, hib, orient=0):
        self._check(self.lib.cfd_connect(self.ctx, a, fa, int2(loa), int2(hia), b, fb, int2(lob), int2(hib), orient))

    def finalize_and_bind(self):
        nbytes = ctypes.c_size_t()
        self._check(self.lib.cfd_finalize(self.ctx, ctypes.byref(nbytes)))
        # torch's caching allocator hands out 512-byte aligned blocks
        self.workspace = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=self.device)
        self._check(self.lib.cfd_bind_workspace(self.ctx, dptr(self.workspace), nbytes.value))
        self.ncells = self.query("ncells")

    # -- layout helpers (marshalling) ----------------------------------------
    def pack(self, arrays):
        """Per-block (nvar, [nk,] nj, ni) arrays -> packed (nvar, ncells) device tensor."""
        flat = [torch.as_tensor(np.asarray(a), dtype=F64).reshape(self.nvar, -1) for a in arrays]
        return torch.cat(flat, dim=1).to(self.device).contiguous()

    def unpack(self, packed):
        out, off = [], 0
        for (ni, nj, nk) in self.block_shapes:
            n = ni * nj * nk
            shape = (self.nvar, nk, nj, ni) if self.dim == 3 else (self.nvar, nj, ni)
            out.append(packed[:, off:off + n].reshape(shape))
            off += n
        return out

    # -- entry points ----------------------------------------------------------
    def set_state(self, Q):
        Q = Q.to(device=self.device, dtype=F64).contiguous()
        self._check(self.lib.cfd_set_state(self.ctx, dptr(Q)))
        self.has_state = True

    def set_state_primitive(self, q):
        q = q.to(device=self.device, dtype=F64).contiguous()
        self._check(self.lib.cfd_set_state_primitive(self.ctx, dptr(q)))
        self.has_state = True

    def get_state(self):
        Q = torch.empty((self.nvar, self.ncells), dtype=F64, device=self.device)
        self._check(self.lib.cfd_get_state(self.ctx, dptr(Q)))
        return Q

    def residual(self, out=None):
        R = torch.empty((self.nvar, self.ncells), dtype=F64, device=self.device) if out is None else out
        self._check(self.lib.cfd_residual(self.ctx, dptr(R)))
        return R

    def residual_norms(self):
        """(R, per-variable RMS norms of R) at the current state."""
        R = torch.empty((self.nvar, self.ncells), dtype=F64, device=self.device)
        N = torch.empty(self.nvar, dtype=F64, device=self.device)
        self._check(self.lib.cfd_residual_norms(self.ctx, dptr(R), dptr(N)))
        return R, N

    def enable_limiter_freezing(self, enable=True):
        """Reserve the frozen-limiter arrays (before finalize)."""
        self._check(self.lib.cfd_enable_limiter_freezing(self.ctx, 1 if enable else 0))

    def freeze_limiter(self, freeze=True):
        """Freeze the limiter at the current state (True) or return to the live limiter."""
        self._check(self.lib.cfd_freeze_limiter(self.ctx, 1 if freeze else 0))

    def time_step(self):
        dt = torch.empty(1, dtype=F64, device=self.device)
        self._check(self.lib.cfd_time_step(self.ctx, dptr(dt)))
        return dt

    def rk_step(self, nsteps=1, dt_out=None):
        self._check(self.lib.cfd_rk_step(self.ctx, int(nsteps), None if dt_out is None else dptr(dt_out)))

    def padded_primitives(self):
        n = ctypes.c_size_t()
        self._check(self.lib.cfd_padded_size(self.ctx, ctypes.byref(n)))
        out = torch.empty(n.value, dtype=F64, device=self.device)
        self._check(self.lib.cfd_padded_primitives(self.ctx, dptr(out)))
        res, off = [], 0
        for (ni, nj, nk) in self.block_shapes:
            shape = (self.nvar, nk + 4, nj + 4, ni + 4) if self.dim == 3 else (self.nvar, nj + 4, ni + 4)
            cnt = int(np.prod(shape))
            res.append(out[off:off + cnt].reshape(shape))
            off += cnt
        return res

    def set_nodes(self, nodes_packed):
        nodes_packed = nodes_packed.to(device=self.device, dtype=F64).contiguous()
        self._check(self.lib.cfd_set_nodes(self.ctx, dptr(nodes_packed)))

    def set_bc_params(self, patch_id, params):
        arr = (ctypes.c_double * 5)(*([float(x) for x in params] + [0.0] * (5 - len(params))))
        self._check(self.lib.cfd_set_bc_params(self.ctx, patch_id, ctypes.cast(arr, capi._DP)))

    def set_exec(self, mode="batched", use_graph=True):
        m = {"batched": capi.EXEC_BATCHED, "per_block": capi.EXEC_PER_BLOCK,
             "persistent": capi.EXEC_PERSISTENT}[mode]
        self._check(self.lib.cfd_set_exec(self.ctx, m, 1 if use_graph else 0))

    def set_ghost_exchange(self, mode="direct"):
        m = {"direct": capi.GHOSTS_DIRECT, "packed": capi.GHOSTS_PACKED}[mode]
        self._check(self.lib.cfd_set_ghost_exchange(self.ctx, m))

    def set_variant(self, v):
        self._check(self.lib.cfd_set_variant(self.ctx, int(v)))

    def autotune(self, reps=5):
        ch = ctypes.c_int()
        self._check(self.lib.cfd_autotune(self.ctx, int(reps), ctypes.byref(ch)))
        return ch.value

    def profile(self, enable=True):
        self._check(self.lib.cfd_profile(self.ctx, 1 if enable else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        self._check(self.lib.cfd_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- adjoint -------------------------------------------------------------
    def enable_adjoint(self, enable=True):
        self._check(self.lib.cfd_enable_adjoint(self.ctx, 1 if enable else 0))

    def _zeros(self, n):
        return torch.zeros(n, dtype=F64, device=self.device)

    def nnodes(self):
        return self.query("nnodes")

    def residual_vjp(self, Rbar, nodes=False, inflow=False):
        Rbar = Rbar.to(device=self.device, dtype=F64).contiguous()
        Qbar = torch.empty((self.nvar, self.ncells), dtype=F64, device=self.device)
        Xbar = torch.empty((self.dim, self.nnodes()), dtype=F64, device=self.device) if nodes else None
        Tbar = torch.empty((max(self.ninflow, 1), self.nvar), dtype=F64, device=self.device) if inflow else None
        self._check(self.lib.cfd_residual_vjp(self.ctx, dptr(Rbar), dptr(Qbar), None if Xbar is None else dptr(Xbar),
                                              None if Tbar is None else dptr(Tbar)))
        return Qbar, Xbar, Tbar

    @property
    def ninflow(self):
        return sum(1 for k in self.patch_kinds if k == "sup_inflow")

    def inflow_slot(self, patch_id):
        """Row of a supersonic-inflow patch in the inflow cotangent arrays
        (the inflow patches in patch-id order)."""
        inflow = sorted(pid for pid, k in zip(self.patch_ids, self.patch_kinds) if k == "sup_inflow")
        if patch_id not in inflow:
            raise ValueError("patch %d is not a supersonic-inflow patch" % patch_id)
        return inflow.index(patch_id)

    def adjoint_reset(self):
        self._check(self.lib.cfd_adjoint_reset(self.ctx))

    def rk_step_vjp(self, Qbar):
        """In place: Qbar holds dJ/dQ^{n+1} on entry and dJ/dQ^n on return."""
        assert Qbar.is_contiguous() and Qbar.dtype == F64
        self._check(self.lib.cfd_rk_step_vjp(self.ctx, dptr(Qbar)))
        return Qbar

    def stage_record_buffer(self, nsteps):
        """Device buffer for the stage states of `nsteps` recorded steps (taken
        from this solver's pool of released buffers when one is large enough)."""
        per = self.state_bytes() * self.stages
        need = nsteps * per
        for n, buf in enumerate(self._record_pool):
            if buf.numel() >= need:
                return self._record_pool.pop(n), per
        return torch.empty(need, dtype=torch.uint8, device=self.device), per

    def release_record_buffer(self, buf):
        """Return a buffer from stage_record_buffer to the pool."""
        if buf is not None:
            self._record_pool.append(buf)

    def rk_step_record(self, slots):
        """One step that leaves its ghost-filled stage inputs in `slots`
        (a uint8 device tensor of stages * state_bytes())."""
        assert slots.numel() >= self.state_bytes() * self.stages
        self._check(self.lib.cfd_rk_step_record(self.ctx, dptr(slots)))

    def rk_step_vjp_recorded(self, slots, Qbar):
        """rk_step_vjp over the stage states of a recorded step."""
        assert Qbar.is_contiguous() and Qbar.dtype == F64
        assert slots.numel() >= self.state_bytes() * self.stages
        self._check(self.lib.cfd_rk_step_vjp_recorded(self.ctx, dptr(slots), dptr(Qbar)))
        return Qbar

    def objective_wall_pressure(self, with_grad=True):
        J = torch.empty(1, dtype=F64, device=self.device)
        Qbar = torch.empty((self.nvar, self.ncells), dtype=F64, device=self.device) if with_grad else None
        self._check(self.lib.cfd_objective_wall_pressure(self.ctx, dptr(J), None if Qbar is None else dptr(Qbar)))
        return J, Qbar

    def adjoint_result(self, nodes=True, inflow=True):
        Xbar = torch.empty((self.dim, self.nnodes()), dtype=F64, device=self.device) if nodes else None
        Tbar = torch.empty((max(self.ninflow, 1), self.nvar), dtype=F64, device=self.device) if inflow else None
        self._check(self.lib.cfd_adjoint_result(self.ctx, None if Xbar is None else dptr(Xbar),
                                                None if Tbar is None else dptr(Tbar)))
        return Xbar, Tbar

    def uniform_state_vjp(self, theta, Qbar):
        th = (ctypes.c_double * 5)(*([float(x) for x in theta] + [0.0] * (5 - len(theta))))
        out = torch.empty(self.nvar, dtype=F64, device=self.device)
        self._check(self.lib.cfd_uniform_state_vjp(self.ctx, ctypes.cast(th, capi._DP), dptr(Qbar.contiguous()),
                                                   dptr(out)))
        return out

    def state_bytes(self):
        n = ctypes.c_size_t()
        self._check(self.lib.cfd_state_size(self.ctx, ctypes.byref(n)))
        return n.value

    def save_state(self, buf=None):
        if buf is None:
            buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._check(self.lib.cfd_save_state(self.ctx, dptr(buf)))
        return buf

    def load_state(self, buf):
        self._check(self.lib.cfd_load_state(self.ctx, dptr(buf)))
        self.has_state = True

    def pack_nodes(self, node_arrays):
        """Per-block node arrays (dim, ...) -> concatenated (dim, nnodes) device tensor."""
        flat = [torch.as_tensor(np.asarray(a), dtype=F64).reshape(self.dim, -1) for a in node_arrays]
        return torch.cat(flat, dim=1).to(self.device).contiguous()

    def query(self, what):
        v = ctypes.c_longlong()
        self._check(self.lib.cfd_query(self.ctx, capi.Q[what], ctypes.byref(v)))
        return v.value

    def close(self):
        if self.ctx:
            self.lib.cfd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
