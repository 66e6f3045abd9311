"""MI355X-native discretised 2->2 elastic collision operator (arXiv 2607.00755).

* ``kxg``     -- binding of the C-ABI library libkxg.so (HIP kernels for gfx950)
* ``inputs``  -- seeded synthetic workloads
* ``serving`` -- continuous-batching request loop over the library
* ``build``   -- in-tree build of libkxg.so
"""
__all__ = ["kxg", "inputs", "serving", "build"]
