"""torch.autograd wrapper of the compiler: per-channel noise rates in,
hyperedge probabilities out, with the hand-written adjoint of stage 2.

The hyperedge structure (which faults form each class) depends only on the
circuit; it is fixed by one compile and then reused, so the forward pass is
the Eq. 3 merge at the new rates and the backward pass is
dL/dr_c = sum_{i in c} dp_i/dr_c * prod_{j in class(i), j != i} (1 - 2 p_j) * dL/dq_class(i).
Both run on the device through the C ABI (gp_aggregate,
gp_aggregate_backward) on torch's current stream, with the rates, q and the
gradients in device memory; torch only allocates the tensors.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import _gp
from .api import Driver, Hypergraph


class HypergraphFunction:
    """Differentiable map rates -> hyperedge probabilities for one circuit.

    `compile(rates)` fixes the structure (a full compile); calling the object
    on a float64 tensor of rates (on the driver's device) returns the
    probability of every hyperedge in the order of `structure`. The backward
    pass uses the rates its forward pass saw, and refuses to run once a later
    compile on the driver has replaced the structure."""

    def __init__(self, driver: Driver, circuit: str):
        self.driver = driver
        self.circuit = circuit
        self.structure: Optional[Hypergraph] = None
        self.structure_id = 0
        self.n_channels = 0

    def compile(self, rates: Sequence[float]) -> Hypergraph:
        self.structure = self.driver.compile_hypergraph(self.circuit, np.asarray(rates, dtype=np.float64))
        self.structure_id = _gp.gp_structure_id(self.driver.handle)
        self.n_channels = int(self.driver.info()["n_channels"])
        return self.structure

    def _check_structure(self) -> None:
        if self.structure is None:
            raise RuntimeError("compile(rates) first: the hyperedge structure is not fixed yet")
        if _gp.gp_structure_id(self.driver.handle) != self.structure_id:
            raise RuntimeError("the driver compiled another circuit since this structure was fixed; "
                               "call compile() again")

    def __call__(self, rates):
        import torch

        fn = self

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, r):
                if fn.structure is None:
                    fn.compile(r.detach().to("cpu", torch.float64).numpy())
                fn._check_structure()
                if r.device.type != "cuda" or r.dtype != torch.float64:
                    raise TypeError("rates must be a float64 tensor on the GPU")
                r = r.detach().contiguous()
                if r.numel() != fn.n_channels:
                    raise ValueError(f"{r.numel()} rates for {fn.n_channels} channels")
                q = torch.empty(len(fn.structure), dtype=torch.float64, device=r.device)
                stream = torch.cuda.current_stream(r.device).cuda_stream
                _gp.gp_aggregate(fn.driver.handle, r.data_ptr(), r.numel(), q.data_ptr(), q.numel(), stream)
                ctx.save_for_backward(r)
                ctx.structure_id = fn.structure_id
                return q

            @staticmethod
            def backward(ctx, grad_q):
                (r,) = ctx.saved_tensors
                if _gp.gp_structure_id(fn.driver.handle) != ctx.structure_id:
                    raise RuntimeError("the driver's hyperedge structure changed between forward and backward")
                gq = grad_q.detach().to(r.device, torch.float64).contiguous()
                gr = torch.empty_like(r)
                stream = torch.cuda.current_stream(r.device).cuda_stream
                _gp.gp_aggregate_backward(fn.driver.handle, r.data_ptr(), r.numel(), gq.data_ptr(), gq.numel(),
                                          gr.data_ptr(), stream)
                return gr

        return _Fn.apply(rates)
