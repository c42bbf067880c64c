"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  No finite-volume arithmetic lives here."""
from .configs import (BASE_SEED, BC, DYNAMIC_WALL, Diffusion, INFLOW_FROUDE, INFLOW_UNIFORM, OUTFLOW_HQ,  # noqa: F401
                      OUTFLOW_UNIFORM, OUTFLOW_WEIR, OUTFLOW_ZEROGRAD, SRC_AVAILABLE, SRC_DISCHARGE,
                      SRC_EXACT, SRC_INFINITY, SRC_INTENSITY, WALL, ZHYDROGRAPH, Morpho, Scenario, Source,
                      dam_break, ensemble_member, ensemble_sizes, lake_at_rest, level_basin, rng,
                      pool_request, serving_pool, serving_request, serving_trace, t5_rarefactions,
                      t6_three_humps, tiny_random, valley_flood, wet_snapshot)
