"""MI355X engine for the batched Hamiltonian slice sampling walk of
gradient-guided nested sampling (arXiv:2312.03911).

Submodules are imported lazily so that `inputs` and `exact` can be used on a
machine without the HIP runtime:
  inputs   seeded synthetic workloads (RunConfig)
  exact    closed-form evidences of those workloads
  _lib     ctypes binding of libggns.so (the C ABI in include/ggns.h)
  engine   device-memory plumbing and the run loop on top of the C ABI
  autograd torch.autograd.Function wrappers around the adjoint kernels
  tuner    tile-shape autotuner
"""
__all__ = ["inputs", "exact"]
