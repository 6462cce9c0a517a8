"""MI355X-native LArTPC signal simulation (rasterisation + FFT convolution) in HIP for gfx950.

Submodules:
  wct    - ctypes binding of libwct.so (the C ABI declared in include/wct.h); importing it
           loads the library and fails loudly when it is not built.
  torch_ops - torch.autograd.Function and tensor-level helpers over the binding.
  synth  - seeded synthetic workloads (depositions, geometries, responses).
  build  - compiles libwct.so for gfx950.
"""
__all__ = ["wct", "synth", "build"]
