"""FP64 CPU oracle for the NanoGS simplification hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
runs this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.
"""
from .nanogs_oracle import (  # noqa: F401
    crn_block, splitmix64, activate, rotation_matrix, covariance,
    knn, union_edges, edge_costs, greedy_pairs, mpmm, merge_pairs,
    scale_rot_from_cov, quat_from_rotation, simplify, deactivate,
    opacity_prune, State, mass, merge_parents, gauss_kl, COST_MC, COST_MC_STRAT, COST_BOUND,
    local_refresh, pass_budget,
)
