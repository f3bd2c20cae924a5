"""Seeded synthetic inputs shared by the oracle tests, the device tests and the bench.

This package draws particle trajectories and observation grids only; it holds none of
the radiation arithmetic (amplitudes, phases, form factors, sums)."""
from .betatron import (C_LIGHT, FIELDS, Bunch, draw_bunch, stack_steps, circular_orbit,
                       replicate, flatten, round_to)
from .configs import (SHAPES, Workload, TINY, SINGLE, PRECISION, CONFIGS, MultiBunch,
                      batched_uneven, serving_bunches, poisson_trace, host_workers, direction_grid, omega_grid,
                      block_log_omegas, Fig3Analogue)
