"""Seeded synthetic workloads (rotated boxes, convex polygons, 3D scenes).

This module only draws inputs: it holds none of the IoU method's arithmetic,
and both the GPU library's callers and the oracle's tests read its output.
"""
from .workloads import (  # noqa: F401
    WORKLOADS, boxes_to_quads, c1_pairs, c2_matrix, c3_boxes, c3_intersect, c3_pairs, c4_polygons,
    c4_simple, c5_scenes, degenerate_stress, get, random_simple,
)
