"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds configurations and input generators only; it performs no
step of the reconstruction method.
"""
from .configs import (Config, CONFIGS, cfg_tiny, cfg_paper, cfg_precision, cfg_cnn, cfg_stream,
                      with_frames, with_angles, with_blocks)
from .medium import Medium, make_medium, point_medium
from .labels import plane_positions
from .records import RECORD_DTYPE, plane_records

__all__ = ["Config", "CONFIGS", "cfg_tiny", "cfg_paper", "cfg_precision", "cfg_cnn",
           "cfg_stream", "with_frames", "with_angles", "with_blocks", "Medium", "make_medium",
           "point_medium", "plane_positions", "RECORD_DTYPE", "plane_records"]
