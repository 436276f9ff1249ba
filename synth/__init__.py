"""Seeded synthetic stereo inputs shared by the oracle's and the GPU path's tests."""
from .scenes import (aerial, batch_specs, jitter, slanted_planes,  # noqa: F401
                     value_noise)
from .configs import workload  # noqa: F401
