"""Seeded synthetic inputs and workload descriptions.

This module holds data only: workload sizes, material constants and the
seeded random fields that stand in for the states of the paper's
single-edge-notched simulations (Section 5).  It contains none of the
method's arithmetic (no residual, no operator, no solver step), so the
CPU oracle and the HIP path can both draw their inputs from it without
sharing any computation.
"""
from .configs import CONFIGS, Config, config_by_name, level_list  # noqa: F401
from .fields import make_inputs, node_coords  # noqa: F401
