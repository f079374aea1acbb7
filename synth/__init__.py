"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Nothing here implements the estimation method; see generator.py."""
from .generator import Scan, make_scan, as_device_input, centred_fft, centred_ifft, grid_positions  # noqa: F401
from . import workloads  # noqa: F401
