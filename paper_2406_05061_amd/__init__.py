"""MI355X-native (gfx950) hot path of progressive entropic optimal transport.

The compute lives in libprogot.so (hand-written HIP kernels behind the C ABI
of include/progot.h); this package is its Python binding.
"""
from .progot import (  # noqa: F401
    Clouds, EpsSchedule, PotError, Server, ProgOTInfo, SinkhornInfo, coupling_metrics, diag_metrics,
    entropic_map, eps_schedule, header_symbols, lib, sinkhorn_divergence,
    marginal_check, prepare_clouds, timing_enable, timing_read, progot_map, progot_solve, sinkhorn_solve, status_string,
    to_device, version, workspace_bytes,
)
