"""Seeded synthetic workloads for the hypothesis-tested progressive kernel estimator.

This package only draws inputs (hit points, light vertices, radius parameters). It holds none of the
estimator's own arithmetic, so both the CPU oracle and the GPU path may consume its arrays.
"""
from .generators import (  # noqa: F401
    Params, KernelSet, PhotonBatch, Workload,
    config0, config1, config2, config4, box_scene, small_config0, uniform_config,
)
