"""Seeded synthetic phantoms: the inputs shared by the FP64 oracle and the HIP path.

This package produces problem *inputs* only -- a voxel grid, structure labels,
per-structure prescriptions, coplanar beams cut into 5 mm beamlets, and the
beamlet dose-deposition matrix D_ij (Section 2.1, eq. 2 defines D_ij as the
dose to voxel j from beamlet i at unit intensity).  It holds none of the
optimisation method's arithmetic: no dose products, objective, gradient,
pricing or master solve lives here.

The pencil-beam kernel that fills D_ij is a stand-in for the GPU dose engine
the paper takes its coefficients from (Section 1 and Section 2.1); its form is
stated in :mod:`phantom.generator`.
"""
from .generator import Phantom, make_phantom, CONFIGS  # noqa: F401
