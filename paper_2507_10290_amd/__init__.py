"""MI355X consensus-ADMM trajectory sweep (TOP, arXiv 2507.10290).

* ``binding``   -- ctypes binding of the HIP library ``libtop.so`` (C ABI in include/top.h)
* ``workloads`` -- seeded synthetic inputs of the benchmark workloads
* ``build``     -- in-tree hipcc build of the library for gfx950
"""
from .binding import TopError, TopProblem, lib, top_cost_fn  # noqa: F401

__all__ = ["TopProblem", "TopError", "lib", "top_cost_fn"]
