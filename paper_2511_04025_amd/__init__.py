"""MI355X-native periodic voxel homogenization of charge-parametrized shells.

Submodules (imported on demand so that ``workloads`` stays free of the GPU
stack): ``binding`` (ctypes over libshellhom), ``api`` (entry points),
``autograd`` (torch.autograd.Function over the adjoint), ``serving`` (the
continuous-batching engine), ``build`` (compiles the HIP library in-tree),
``workloads`` (seeded synthetic inputs).
"""
__all__ = ["api", "autograd", "binding", "build", "serving", "workloads"]
