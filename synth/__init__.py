"""Seeded synthetic scan generation shared by the oracle checks, the GPU tests and the benchmark."""
from .scans import (C0, DT, Grid, Scan, c1_scan, c2_scan, c3_scan, c4_scan, c4_shape,  # noqa: F401
                    cube_grid, hemisphere_antennas, make_scan, ms_scan, point_scan, pulse, random_scan,
                    random_scan_ms, ring_antennas, square_grid, synthesize, synthesize_ms)
from .rng import SplitMix64, gaussian_noise, philox4x32_10  # noqa: F401
