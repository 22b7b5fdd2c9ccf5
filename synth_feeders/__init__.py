"""Seeded synthetic three-phase radial feeders (inputs only).

This package builds the inputs of the aggregation search: topology, phase
sets, per-edge admittance blocks, per-snapshot constant-PQ loads, the
eligible-node mask and the segment ids.  It contains none of the search's
arithmetic (no power flow, no Kron reduction, no scoring); both the HIP
library and the CPU oracle consume what it produces.
"""
from .feeders import CONFIGS, FeederConfig, make_feeder, dfs_preorder, hourly_feeder, extreme_scenarios

__all__ = ["CONFIGS", "FeederConfig", "make_feeder", "dfs_preorder", "hourly_feeder", "extreme_scenarios"]
