"""Seeded synthetic inputs (meshes, boundary data, states) shared by the CPU
oracle, the tests and the benchmark.  Geometry and bookkeeping only."""
from .cases import Case, build, cube_lid, channel2, pipe, PIPE_SIZES  # noqa: F401
