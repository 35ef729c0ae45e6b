"""Seeded synthetic workloads: circuit text generators and per-channel noise rates.

This package produces inputs only. It contains none of the compiler's arithmetic
(no propagation, no probability split, no merging), so both the HIP path and the
CPU oracle may consume what it generates without sharing any method code.
"""

from .circuits import (  # noqa: F401
    Circuit,
    rotated_surface_code_memory,
    paper_noise,
    repetition_code_memory,
    bivariate_bicycle_memory,
    bit_flip_code_fig1,
    mirror_circuit,
)
from .concatenated import (  # noqa: F401
    iceberg_pairing,
    iceberg_pairing_violations,
    iceberg_surface_branch,
    iceberg_surface_batch,
)
from .rates import splitmix64_uniform, log_uniform_rates  # noqa: F401
from .loss import logit_loss  # noqa: F401
