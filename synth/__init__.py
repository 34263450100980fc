"""Seeded synthetic graphs and source lists (inputs only; no step of the method)."""
from .graphs import *  # noqa: F401,F403
from .graphs import build  # noqa: F401
