"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench."""
from .systems import *  # noqa: F401,F403
