"""Seeded synthetic inputs for Aggregate Risk Analysis (ARA).

This package only draws random inputs: Year Event Tables, dense Event Loss
Tables and the financial terms attached to them.  It holds none of the
method's arithmetic (no lookups, no terms applied, no sums of losses), so it
can feed both the CPU oracle and the GPU library without coupling them.
"""

from .generators import (  # noqa: F401
    SEED_BASE,
    YET,
    ELTPool,
    Layer,
    Workload,
    make_yet,
    make_timestamps,
    make_elt_pool,
    elt_terms_from_losses,
    make_config,
    make_tiny_yet,
    layer_library,
    portfolio_programs,
    CONFIG_NAMES,
)
