"""DRGraph layout hot path on MI355X (gfx950).

* ``gen``      -- seeded synthetic input graphs (canonical CSR)
* ``drgraph``  -- Python binding of libdrgraph.so (the HIP library)
* ``build``    -- compiles libdrgraph.so with hipcc for gfx950
"""
from . import gen  # noqa: F401

__all__ = ["gen"]
