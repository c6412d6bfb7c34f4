"""CPU oracle for Aggregate Risk Analysis -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg use this package.  The GPU library never imports, links or calls it, and
it shares no code with the GPU library: both sides receive the same seeded
inputs from ``workloads`` and nothing else.

Parity status of each function is stated in its docstring ("pinned by" lists
the checks in tests/test_oracle_pins.py that tie it to the paper or to
mathematics rather than to itself).
"""

from .reference import (  # noqa: F401
    run_layer,
    run_layer_python,
    run_layer_numpy,
    occurrence_catalogue,
    event_nets,
    portfolio,
    event_nets_python,
    lookups,
    tail_count,
    risk_metrics,
    grad_counts,
    gradients,
    exact_sum,
    max_threads,
)
