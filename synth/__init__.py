"""Seeded synthetic inputs shared by the oracle tests and the GPU library tests.

Nothing here performs any step of the receive pipeline; it only lays out probes,
scanlines and scatterers and simulates the channel data a probe would record.
"""
from .geometry import (Geometry, ScanGrid, HANN, RECT, linear_2d, matrix_3d, config_small_2d,
                       config_multiline_2d, config_volume_3d, config_tiny, stream_mix,
                       config_planewave_2d, config_overlap_2d)
from . import phantom, rfsim
