"""Seeded synthetic inputs for TSDF-Sampling workloads.

This package only generates inputs: analytic scenes and their exact ray
depths (standing in for the depth a trained network would render, Eq. 2),
pinhole / equirectangular cameras, seeded MLP parameters and the workload
configurations.  It holds none of the method's arithmetic (no voxel
traversal, no TSDF update, no sampling, no rendering), so both the CPU
oracle and the GPU path can consume its arrays without sharing code.
"""
from .scenes import Scene, Sphere, Box, Room, pinhole_rays, equirect_rays  # noqa: F401
from .configs import get_config, CONFIG_NAMES  # noqa: F401
