"""Seeded synthetic fragment pairs for global registration tests and benchmarks.

The paper evaluates on pairwise-registration fragments fused from augmented
ICL-NUIM sequences (Sec. IV, Table 1).  Those fragments are not available
here, so this module builds stand-ins with the same structure: indoor
surfaces (planes, boxes, cylinders, spheres) sampled at sensor resolution,
cropped into two partially overlapping fragments, perturbed by Gaussian noise,
and separated by a known rigid transform.

This module holds no arithmetic of the registration method itself (no
neighbourhoods, normals estimation, descriptors, matching, or pose solving).
It only produces inputs, shared by the CPU oracle and the GPU path.

Every array is float32 structure-of-arrays: a cloud is a (6, N) array with rows
x, y, z, nx, ny, nz.  ``T_gt`` is a float64 4x4 matrix mapping P into Q's
frame (q ~ R p + t), the output the method should recover.
"""
from .scenes import (  # noqa: F401
    Pair,
    make_pair,
    make_batch,
    random_rigid,
    CONFIG_NAMES,
)
