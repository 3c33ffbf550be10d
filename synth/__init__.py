"""Seeded synthetic electron-microscopy inputs and workload definitions.

This package only produces inputs (images, masks, ground truth) and names the
workload shapes; it holds none of the BPFA arithmetic.  Both the CPU oracle
and the GPU path read their inputs from here, so they see identical data.

The paper's STEM / SEM frames are not available; the generators stand in for
them with atom-column lattices of Gaussian blobs under Poisson counting noise,
normalised to [0, 1], and uniformly random sampling masks.
"""
from .lattice import (WORKLOADS, Workload, make_frame, make_mask, make_serving_frame,  # noqa: F401
                      workload)
