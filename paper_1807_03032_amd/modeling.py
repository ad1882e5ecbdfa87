"""Forward modelling, adjoint and gradient with respect to m for the isotropic
operator, with checkpointed forward recomputation, and a torch.autograd
wrapper.

Every stencil, injection, interpolation and imaging-condition step runs in the
HIP kernels of libfdw.so (through the C ABI in fdw.py); this module only
orchestrates operators, buffers and the order of the steps.

The adjoint follows from transposing the discrete time loop (the consistency
the paper's Section 3.2 builds in by making injection the adjoint of
interpolation): with nu = (dt^2/m) D^-1 lambda (D = 1 + eta dt/2) the
transposed recurrence is the forward leapfrog run backwards in time, driven by
the residual traces injected at the receivers (inside the damping division),
with the source-side output sampled from D nu.  The gradient of
J(m) = sum_t <d(t), rec(t)> is the zero-lag imaging condition
  dJ/dm = -sum_t nu(t+1) [(u(t+1) - 2u(t) + u(t-1))/dt^2 + eta (u(t+1) - u(t-1))/(2 dt)].
The forward kernels store the bracket (times dt^2) of each step of a segment
as they compute it, and the adjoint kernels fold the product with nu into
their own launches, so a segment's gradient is one forward apply (skipped for
the last segment, whose factors the forward run itself keeps) and one adjoint
call.  With enough device memory the segment is the whole run and nothing is
recomputed.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import fdw


class IsoModeling:
    """One isotropic shot geometry on the GPU: forward, adjoint, gradient.

    shape/extent/origin follow fdw_grid_create; src_coords [nsrc][ndim],
    rec_coords [nrec][ndim]; `checkpoint_every` = K steps between checkpoints
    (each checkpoint keeps two consecutive levels; the gradient keeps the
    imaging factors of one K-step segment).  None: K = nt (no recomputation)
    when the factors of all nt steps fit in `history_fraction` of the free
    device memory, else 50.
    """

    def __init__(self, shape, extent, origin, so: int, dt: float, nt: int, nbl: int, vmax: float, src_coords,
                 rec_coords, device="cuda:0", checkpoint_every: Optional[int] = 50, rc: float = 1e-3,
                 history_fraction: float = 0.9):
        import torch

        self.torch = torch
        self.dev = torch.device(device)
        self.nt, self.dt, self.so = int(nt), float(dt), int(so)
        self.grid = fdw.fdw_grid_create(shape, extent, origin)
        self.lay = fdw.fdw_field_layout(self.grid, so)
        E = self.lay.elems_per_slot
        self.E = E
        self.src_coords = np.ascontiguousarray(src_coords, dtype=np.float64)
        self.rec_coords = np.ascontiguousarray(rec_coords, dtype=np.float64)
        nsrc, nrec = self.src_coords.shape[0], self.rec_coords.shape[0]
        self.nsrc, self.nrec = nsrc, nrec
        alloc = lambda n: fdw.alloc_field(self.lay, n, self.dev)  # noqa: E731
        self.m = alloc(1)
        self.m.fill_(1.0)
        self.m_fn = fdw.fdw_function_bind(self.grid, "m", self.m.data_ptr(), E, so)
        # forward operator: u, sources -> receivers
        self.u = alloc(3)
        self.u_tf = fdw.fdw_timefunction_bind(self.grid, "u", self.u.data_ptr(), self.u.numel(), so, 2, 3)
        self.q = torch.zeros((nt, nsrc), dtype=torch.float32, device=self.dev)
        self.rec = torch.zeros((nt, nrec), dtype=torch.float32, device=self.dev)
        self.f_src = fdw.fdw_sparse_bind(self.grid, "src", self.src_coords, nt, self.q.data_ptr())
        self.f_rec = fdw.fdw_sparse_bind(self.grid, "rec", self.rec_coords, nt, self.rec.data_ptr())
        # adjoint operator: nu, residuals at the receivers -> samples at the sources
        self.nu = alloc(3)
        self.nu_tf = fdw.fdw_timefunction_bind(self.grid, "nu", self.nu.data_ptr(), self.nu.numel(), so, 2, 3)
        self.d_rev = torch.zeros((nt, nrec), dtype=torch.float32, device=self.dev)
        self.a_out = torch.zeros((nt, nsrc), dtype=torch.float32, device=self.dev)
        self.a_src = fdw.fdw_sparse_bind(self.grid, "adj_src", self.rec_coords, nt, self.d_rev.data_ptr())
        self.a_rec = fdw.fdw_sparse_bind(self.grid, "adj_rec", self.src_coords, nt, self.a_out.data_ptr())
        # torch loads a kernel's code on its first use in the process (about
        # 50 ms for the time reversal): reverse a tiny tensor once here, so that
        # adjoint() and gradient() spend their time on their own work
        torch.flip(self.d_rev[:2], dims=[0])

        def desc(u_tf, src, rec, mode):
            d = fdw.fdw_op_desc()
            d.kind, d.space_order, d.dt, d.nbl, d.damp_rc, d.vmax = fdw.FDW_ISO, so, dt, nbl, rc, vmax
            d.u, d.m, d.src, d.rec, d.mode = u_tf, self.m_fn, src, rec, mode
            return d

        self.fwd = fdw.fdw_operator_create(desc(self.u_tf, self.f_src, self.f_rec, fdw.FDW_FORWARD))
        self.adj = fdw.fdw_operator_create(desc(self.nu_tf, self.a_src, self.a_rec, fdw.FDW_ADJOINT))
        self.grad = alloc(1)
        if checkpoint_every is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            checkpoint_every = self.nt if self.nt * E * 4 <= history_fraction * free else 50
        self.K = min(max(1, int(checkpoint_every)), self.nt)
        self.ncp = (nt + self.K - 1) // self.K
        # checkpoints [ncp][2 slots]: levels (kK - 1, kK); imaging factors of the
        # steps t0 .. t0 + K - 1 of one segment.  Allocated (and first touched:
        # fresh device memory may be cleared on first use) with the model, so
        # that runs reuse them
        self.cp = torch.zeros(self.ncp * 2 * E, dtype=torch.float32, device=self.dev)
        self.hist = torch.zeros(self.K * E, dtype=torch.float32, device=self.dev)
        # changes with every new m and every forward run: the checkpoints (and
        # q) a gradient uses belong to the state of that number
        self.state_id = 0
        self.hist_seg = None  # (segment, state) whose factors self.hist holds
        self.cp_state = None  # state the checkpoints belong to

    # ------------------------------------------------------------------ data
    def stream(self):
        return self.torch.cuda.current_stream(self.dev).cuda_stream

    def set_m(self, m):
        """m: logical squared slowness, numpy (nz, [ny,] nx) or a tensor of that shape."""
        t = self.torch.as_tensor(m, dtype=self.torch.float32, device=self.dev)
        fdw.slot_view(self.m, self.lay, 0).copy_(t)
        self.state_id += 1

    def _slot(self, buf, k):
        return buf[k * self.E:(k + 1) * self.E]

    def _ptr(self, buf, k):
        return buf.data_ptr() + 4 * k * self.E

    # --------------------------------------------------------------- forward
    def forward(self, q, checkpoints: bool = True):
        """Receiver traces [nt][nrec] of the sources q [nt][nsrc] from zero initial levels."""
        torch = self.torch
        self.state_id += 1
        self.q.copy_(torch.as_tensor(q, dtype=torch.float32, device=self.dev).reshape(self.nt, self.nsrc))
        self.u.zero_()
        self.rec.zero_()
        fdw.fdw_operator_set_save(self.fwd, None)
        fdw.fdw_operator_set_imaging_save(self.fwd, None)
        self.hist_seg = None
        for k in range(self.ncp):
            t0, t1 = k * self.K, min((k + 1) * self.K, self.nt)
            last = checkpoints and k == self.ncp - 1
            if checkpoints:  # levels t0 - 1 and t0 live in slots (t0 - 1) % 3 and t0 % 3
                self._slot(self.cp, 2 * k).copy_(self._slot(self.u, (t0 + 2) % 3))
                self._slot(self.cp, 2 * k + 1).copy_(self._slot(self.u, t0 % 3))
            if last:  # the gradient starts with this segment: keep its imaging factors now
                fdw.fdw_operator_set_imaging_save(self.fwd, self.hist.data_ptr(), t1 - t0, t0)
            fdw.fdw_operator_apply(self.fwd, t0, t1 - 1, self.stream())
            if last:
                fdw.fdw_operator_set_imaging_save(self.fwd, None)
                self.hist_seg = (k, self.state_id)
        if checkpoints:
            self.cp_state = self.state_id
        return self.rec.clone()

    # --------------------------------------------------------------- adjoint
    def adjoint(self, d):
        """F^T d: [nt][nrec] residual traces -> [nt][nsrc]."""
        torch = self.torch
        d = torch.as_tensor(d, dtype=torch.float32, device=self.dev).reshape(self.nt, self.nrec)
        self.d_rev.copy_(torch.flip(d, dims=[0]))
        self.nu.zero_()
        self.a_out.zero_()
        fdw.fdw_operator_apply(self.adj, 0, self.nt - 1, self.stream())
        return torch.flip(self.a_out, dims=[0]).clone()

    # -------------------------------------------------------------- gradient
    def gradient(self, d, q=None):
        """dJ/dm for J(m) = sum_t <d(t), rec(t)>, rec the traces of the last
        forward() (or of q, recomputed with checkpoints).  Returns the logical
        gradient as a tensor."""
        torch = self.torch
        if q is not None or self.cp_state != self.state_id:
            self.forward(self.q if q is None else q, checkpoints=True)
        d = torch.as_tensor(d, dtype=torch.float32, device=self.dev).reshape(self.nt, self.nrec)
        self.d_rev.copy_(torch.flip(d, dims=[0]))
        self.nu.zero_()
        self.a_out.zero_()
        self.grad.zero_()
        s = self.stream()
        for k in reversed(range(self.ncp)):
            t0, t1 = k * self.K, min((k + 1) * self.K, self.nt)
            if self.hist_seg != (k, self.state_id):
                # recompute the segment from its checkpoint (levels t0 - 1, t0),
                # keeping the imaging factors of its steps t0 .. t1 - 1
                self._slot(self.u, (t0 + 2) % 3).copy_(self._slot(self.cp, 2 * k))
                self._slot(self.u, t0 % 3).copy_(self._slot(self.cp, 2 * k + 1))
                fdw.fdw_operator_set_imaging_save(self.fwd, self.hist.data_ptr(), t1 - t0, t0)
                fdw.fdw_operator_apply(self.fwd, t0, t1 - 1, s)
                fdw.fdw_operator_set_imaging_save(self.fwd, None)
                self.hist_seg = (k, self.state_id)
            # adjoint steps tau = nt - t1 .. nt - 1 - t0 (forward steps t1 - 1 .. t0)
            # with the imaging condition, in one call
            fdw.fdw_gradient_apply(self.adj, self.nt - t1, self.nt - 1 - t0, self.nt, self.hist.data_ptr(), t0,
                                   t1 - t0, self.grad.data_ptr(), s)
        return fdw.slot_view(self.grad, self.lay, 0).clone()

    def close(self):
        if getattr(self, "fwd", None):
            fdw.fdw_operator_destroy(self.fwd)
            fdw.fdw_operator_destroy(self.adj)
            self.fwd = None
            for s in (self.f_src, self.f_rec, self.a_src, self.a_rec):
                fdw.fdw_sparse_destroy(s)
            fdw.fdw_timefunction_destroy(self.u_tf)
            fdw.fdw_timefunction_destroy(self.nu_tf)
            fdw.fdw_function_destroy(self.m_fn)
            fdw.fdw_grid_destroy(self.grid)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wave_forward_function():
    """torch.autograd.Function: traces = F(m) q, with d traces / d m through
    the adjoint-state gradient (checkpointed recomputation)."""
    import torch

    class IsoWaveForward(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, q, model: IsoModeling):
            model.set_m(m)
            traces = model.forward(q, checkpoints=True)
            ctx.model = model
            ctx.state_id = model.state_id
            ctx.save_for_backward(m.detach().clone(), q.detach().clone())
            return traces

        @staticmethod
        def backward(ctx, grad_traces):
            model = ctx.model
            m, q = ctx.saved_tensors
            if model.state_id != ctx.state_id:
                # another forward (or a new m) ran on this model since: restore
                # this call's m and recompute its checkpoints
                model.set_m(m)
                model.forward(q, checkpoints=True)
            g = model.gradient(grad_traces)
            gq = model.adjoint(grad_traces) if ctx.needs_input_grad[1] else None
            return g, gq, None

    return IsoWaveForward
