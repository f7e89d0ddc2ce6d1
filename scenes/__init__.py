"""Seeded synthetic inputs (Gaussians, sensor rigs, rays) shared by the oracle and the library."""
from .synthetic import *  # noqa: F401,F403
