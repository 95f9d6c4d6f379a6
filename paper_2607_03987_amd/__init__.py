"""MI355X-native PAKR planner: parallel AO kinodynamic RRT on gfx950.

``workloads`` builds planning problems; ``pakr`` binds the HIP library
(libpakr.so, C ABI in include/pakr.h).
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "pakr"]
