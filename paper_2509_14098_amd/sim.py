"""Convenience layer over the C interface: a context bound to torch's current
stream, plans with introspection, and an autograd Function whose backward is
the library's adjoint reverse sweep.  Memory comes from torch; every step of
the computation runs in libqsv.so."""
from __future__ import annotations

import torch

from . import binding as B


class Plan:
    def __init__(self, handle, n_qubits):
        self.handle = handle
        self.n = n_qubits
        self.info = B.qsv_plan_info(handle)

    @property
    def n_params(self):
        return self.info["n_params"]

    def partition(self, p, circuit=0, level=0):
        return B.qsv_plan_partition(self.handle, circuit, level, p)

    def partitions(self, circuit=0, level=0):
        out = []
        p = 0
        while True:
            try:
                out.append(self.partition(p, circuit, level))
            except B.QsvError:
                return out
            p += 1

    def refresh(self):
        self.info = B.qsv_plan_info(self.handle)
        return self.info

    def close(self):
        if self.handle is not None:
            B.qsv_plan_destroy(self.handle)
            self.handle = None


class Simulator:
    """One library context on one GPU, following torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = B.qsv_create(device, torch.cuda.current_stream(self.device))

    def _sync_stream(self):
        B.qsv_set_stream(self.ctx, torch.cuda.current_stream(self.device))

    def partition(self, n_qubits, gates, k=0, flags=0, tile=None, circ_offsets=None) -> Plan:
        return Plan(B.qsv_partition(self.ctx, n_qubits, gates, circ_offsets, k, flags, tile), n_qubits)

    def partition_distributed(self, n_qubits, gates, n_global, k=0, flags=0, tile=None) -> Plan:
        """Plan with the distributed level: 2^n_global emulated ranks."""
        return Plan(B.qsv_partition_distributed(self.ctx, n_qubits, gates, n_global, k, flags, tile), n_qubits)

    def specialise(self, plan: Plan) -> float:
        """Compile and load the plan's specialised sweep kernels (host seconds)."""
        secs = B.qsv_plan_specialise(self.ctx, plan.handle)
        plan.info = B.qsv_plan_info(plan.handle)
        return secs

    def specialise_async(self, plan: Plan) -> None:
        """Compile the plan's specialised kernels in the background; applies
        switch to them once loaded (plan.refresh() shows when)."""
        B.qsv_plan_specialise_async(self.ctx, plan.handle)

    def zero_state(self, n_qubits, batch=1):
        psi = torch.zeros((batch, 1 << n_qubits) if batch > 1 else (1 << n_qubits,), dtype=torch.complex64,
                          device=self.device)
        psi.view(batch, -1)[:, 0] = 1.0
        return psi

    def theta(self, values):
        """Parameters as the contiguous float64 device tensor the library reads."""
        if values is None:
            return None
        return torch.as_tensor(values).to(device=self.device, dtype=torch.float64).contiguous()

    def checkpoints(self, plan: Plan):
        nbytes = plan.info["ckpt_bytes"]
        return torch.empty(max(nbytes // 8, 1), dtype=torch.complex64, device=self.device) if nbytes else None

    def apply(self, plan: Plan, psi, theta=None, ckpt=None):
        self._sync_stream()
        B.qsv_apply(self.ctx, plan.handle, self.theta(theta), psi, ckpt)
        return psi

    def expect(self, H, psi, n_qubits, batch=1):
        self._sync_stream()
        out = torch.empty(batch, dtype=torch.float64, device=self.device)
        B.qsv_expect(self.ctx, H, n_qubits, batch, psi, out)
        return out

    def adjoint_grad(self, plan: Plan, H, theta, psi_final=None, ckpt=None):
        self._sync_stream()
        energy = torch.empty(plan.info["n_circuits"], dtype=torch.float64, device=self.device)
        grad = torch.empty(max(plan.n_params, 1), dtype=torch.float64, device=self.device)
        B.qsv_adjoint_grad(self.ctx, plan.handle, H, self.theta(theta), psi_final, ckpt, energy, grad)
        return energy, grad[:plan.n_params]

    def close(self):
        if self.ctx is not None:
            B.qsv_destroy(self.ctx)
            self.ctx = None


class Energy(torch.autograd.Function):
    """E(theta) = <0|C(theta)^dag H C(theta)|0> (float64).  forward runs the
    fused sweeps with partition-boundary checkpoints plus the expectation;
    backward runs the adjoint reverse sweep over the partitions."""

    @staticmethod
    def forward(ctx, theta, sim: Simulator, plan: Plan, H):
        th = theta.detach().to(device=sim.device, dtype=torch.float64).contiguous()
        psi = sim.zero_state(plan.n)
        ckpt = sim.checkpoints(plan)
        sim.apply(plan, psi, th, ckpt)
        e = sim.expect(H, psi, plan.n)[0]
        ctx.save_for_backward(th)
        ctx.sim, ctx.plan, ctx.H, ctx.psi, ctx.ckpt = sim, plan, H, psi, ckpt
        ctx.dtype, ctx.device = theta.dtype, theta.device
        return e.to(theta.device)

    @staticmethod
    def backward(ctx, g_e):
        (th,) = ctx.saved_tensors
        _, grad = ctx.sim.adjoint_grad(ctx.plan, ctx.H, th, ctx.psi, ctx.ckpt)
        return (grad * g_e.to(grad.device)).to(device=ctx.device, dtype=ctx.dtype), None, None, None
