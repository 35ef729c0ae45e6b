"""torch.autograd wrapper of the compiler: per-channel noise rates in,
hyperedge probabilities out, with the hand-written adjoint of stage 2.

The hyperedge structure (which faults form each class) depends only on the
circuit; it is fixed by one compile and then reused, so the forward pass is
the Eq. 3 merge at the new rates and the backward pass is
dL/dr_c = sum_{i in c} dp_i/dr_c * prod_{j in class(i), j != i} (1 - 2 p_j) * dL/dq_class(i).
Both run on the device through the C ABI; torch only carries the tensors.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .api import Driver, Hypergraph


class HypergraphFunction:
    """Differentiable map rates -> hyperedge probabilities for one circuit.

    `compile(rates)` fixes the structure (a full compile); calling the object
    on a float64 tensor of rates returns the probability of every hyperedge
    in the order of `structure`."""

    def __init__(self, driver: Driver, circuit: str):
        self.driver = driver
        self.circuit = circuit
        self.structure: Optional[Hypergraph] = None

    def compile(self, rates: Sequence[float]) -> Hypergraph:
        self.structure = self.driver.compile_hypergraph(self.circuit, np.asarray(rates, dtype=np.float64))
        return self.structure

    def __call__(self, rates):
        import torch

        fn = self

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, r):
                rr = r.detach().to("cpu", torch.float64).numpy()
                if fn.structure is None:
                    fn.compile(rr)
                    hg = fn.structure
                else:
                    hg = fn.driver.refresh_rates(rr)
                return torch.from_numpy(hg.q.copy()).to(r.device)

            @staticmethod
            def backward(ctx, grad_q):
                g = fn.driver.rates_gradient(grad_q.detach().to("cpu", torch.float64).numpy())
                return torch.from_numpy(g).to(grad_q.device)

        return _Fn.apply(rates)
