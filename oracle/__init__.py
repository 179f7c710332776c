"""FP64 CPU oracle for the render + decode hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import it.  It is independent of the GPU
library: no shared kernels, headers, helpers or constants generators.

- ``oracle.raster``: projection, tile binning, compositing and its adjoint
  (plain C, FP64, OpenMP over pixels), plus a tile-free brute force.
- ``oracle.decode_oracle``: dictionary attention, cosine loss with trust region
  and their gradients (numpy FP64).
"""
