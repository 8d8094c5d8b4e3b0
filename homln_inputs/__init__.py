"""Seeded synthetic HoMLN workloads (edge lists only; no method arithmetic)."""
from .configs import HoMLN, make_config, config1, config2, config3, config3_homln, config4, config5, config4_sources  # noqa: F401
from . import generators  # noqa: F401
