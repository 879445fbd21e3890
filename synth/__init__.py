"""Seeded synthetic inputs shared by the oracle and the GPU library (data only)."""
from .scenes import *  # noqa: F401,F403
