"""MI355X-native FDTD as fixed-weight two-layer message passing.

The compute path is the HIP library ``libgemfdtd.so`` (C ABI in
include/gemfdtd.h); ``_lib`` binds it with ctypes, ``sim`` wraps handles,
``autograd`` exposes the adjoint as a torch.autograd.Function, ``workloads``
generates seeded synthetic inputs.  Submodules are imported on demand so
that importing the package touches neither torch nor the GPU.
"""
__all__ = ["_lib", "sim", "workloads", "autograd", "build"]
__version__ = "0.1.0"
