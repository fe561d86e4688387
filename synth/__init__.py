"""Seeded synthetic inputs for the Gaussian-splatting RGB-D renderer.

This module only draws random numbers and builds camera/pose matrices from
look-at parameters.  It holds none of the renderer's arithmetic: both the
GPU library's tests and the CPU oracle consume what it returns.

The paper measures on scanned scenes that are not available, so every
workload here is a synthetic stand-in with the shapes the workload
configurations describe (Gaussian counts, SH degree, spatial layout,
cameras).  All draws use numpy ``Generator(PCG64(seed))`` in a fixed order:
means -> log-scales -> quaternions -> opacity logits -> DC colour ->
higher-order SH.
"""
from .scenes import *  # noqa: F401,F403
