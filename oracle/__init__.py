"""Plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  ``liboracle.so`` is built from ``nlo.c`` (plain C99,
``-ffp-contract=off``); this module marshals numpy arrays into it and adds the
plain dense/CG solves and the L2 error of Sec. 8.
"""
from .binding import (build, OracleProblem, assemble, pairs_of, pair_block, row,
                      load_vector, outer_points, inner_sums, region, census, blocks_range,
                      system_from_full, cg, l2_error, solve_problem, effective_weights, mlp_forward,
                      mlp_backward, cap_moments, cap_candidates, bf16_round, mlp_features)

__all__ = ["build", "OracleProblem", "assemble", "pairs_of", "pair_block", "row",
           "load_vector", "outer_points", "inner_sums", "region", "census", "blocks_range",
           "system_from_full", "cg", "l2_error", "solve_problem", "effective_weights", "mlp_forward",
           "mlp_backward", "cap_moments", "cap_candidates", "bf16_round", "mlp_features"]
