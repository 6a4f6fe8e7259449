"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .posets import *  # noqa: F401,F403
from .posets import __all__  # noqa: F401
