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


def kernel_source_hash() -> str:
    """Short hash of the HIP sources that define the AA step kernels (code
    only: comments and blank lines are dropped) and of the compiler flags;
    ties recorded hardware-counter measurements to the kernel they measured."""
    import hashlib
    import os
    import re
    from .build import FLAGS
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in ("lattice.hpp", "collide.hpp", "cumulant.hpp", "mrt.hpp", "step_impl.hpp",
              "step_q19.hip", "step_q27.hip"):
        with open(os.path.join(here, f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = [ln.split("//")[0].rstrip() for ln in src.splitlines()]
        h.update("\n".join(ln for ln in code if ln.strip()).encode())
    h.update(" ".join(x for x in FLAGS if not x.startswith("-I")).encode())
    return h.hexdigest()[:16]
