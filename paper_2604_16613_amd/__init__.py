"""MI355X just-in-time compiler for decoding hypergraphs (GreenPeas method,
arXiv 2604.16613): circuit text -> detector error model on one gfx950 GPU.

The compute lives in ``libgp.so`` (C ABI in ``include/gp.h``); this package is
its binding. Build it with ``paper_2604_16613_amd._build.build()``.
"""

from . import _gp  # noqa: F401
from ._gp import GpError, GpBounds, GpCircuitInfo  # noqa: F401
from .api import Driver, Hypergraph, Server, get_driver, load_tuning, save_tuning  # noqa: F401
