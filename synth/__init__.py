"""Seeded synthetic inputs for the particle-particle ladder (shared by the
oracle tests and the HIP path; holds none of the method's arithmetic)."""
from .generators import *  # noqa: F401,F403
