"""Seeded synthetic inputs (unit cells, material tables, k-point lists).

This package only draws random numbers and rasterises geometry.  It holds
none of the band-structure arithmetic, so both the CPU oracle and the GPU
harness may import it without sharing any part of the method.
"""
from .cells import *  # noqa: F401,F403
