"""Seeded synthetic inputs shared by the oracle (tests) and the HIP library."""
from . import fields, meshes, scenes  # noqa: F401
from .scenes import Box, Scene, make_config  # noqa: F401
