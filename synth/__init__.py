"""Seeded synthetic input generators (no permutation arithmetic lives here)."""
from .gen import *  # noqa: F401,F403
