"""The differentiation workload's objective (a fit of noise rates to detection
statistics): L = sum_k w_k log(q_k / (1 - q_k)) over the hyperedges, with
seeded weights w_k, and dL/dq_k = w_k / (q_k (1 - q_k)). This is the loss the
workload differentiates through, not part of the compiler's method."""

import numpy as np


def logit_loss(q, w):
    """-> (L, dL/dq) for hyperedge probabilities q and weights w."""
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    return float(np.sum(w * np.log(q / (1.0 - q)))), w / (q * (1.0 - q))
