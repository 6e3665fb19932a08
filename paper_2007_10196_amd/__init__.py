"""MI355X-native sparse-grid WENO5 (Zhu & Zhang, arXiv 2007.10196).

* ``binding``  -- ctypes binding of libsgweno (include/sgweno.h)
* ``solver``   -- Plan / Solver / Batch over PyTorch-owned device memory
* ``serving``  -- continuous-batching serving loop over the batch runtime
* ``autotune`` -- launch-shape tuner for the stage kernel (box target, workgroups per CU)
* ``build``    -- hipcc build of libsgweno.so (gfx950)
"""
__all__ = ["binding", "solver", "serving", "autotune", "build"]
