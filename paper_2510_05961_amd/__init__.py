"""libmsm: multilevel summation electrostatics (MSM with B-spline
interpolation, arXiv 2510.05961) as hand-written HIP kernels for MI355X.

``paper_2510_05961_amd.msm`` is the ctypes binding of the C-ABI library
``libmsm.so`` (plus the torch autograd wrapper); ``workloads`` holds the
seeded synthetic inputs.  Importing the package loads nothing.
"""
__all__ = ["msm", "workloads"]
