"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle."""
from .scenes import *  # noqa: F401,F403
