"""Seeded synthetic inputs shared by the tests, the oracle checks and the
benchmark.  Holds mesh/scene generation only, none of the method."""
from . import meshes, scenes  # noqa: F401
