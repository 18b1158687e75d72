"""MI355X-native sparse (indirect-addressing) AA-pattern lattice Boltzmann path.

Submodules:
  lbm      -- ctypes binding of the C-ABI library ``liblbm.so`` (HIP, gfx950)
  inputs   -- seeded synthetic geometries (label masks); no method arithmetic
  build    -- compiles the HIP library in-tree with hipcc
  server   -- continuous-batching permeability-solve server over ``lbm``
  autotune -- launch-configuration tuner over ``lbm``

Submodules are imported lazily so that the input generators can be used on a
host without a GPU.
"""
__all__ = ["lbm", "inputs", "build", "server", "autotune"]
