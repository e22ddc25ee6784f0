"""Seeded synthetic inputs shared by the oracle and the GPU library.

Meshes, media parameters and random vectors only: nothing here evaluates a
boundary operator, a quadrature rule or an incident field.
"""
from . import meshes, vectors, configs  # noqa: F401
