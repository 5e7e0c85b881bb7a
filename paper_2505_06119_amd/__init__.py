"""Two-site MPS gate update with column-pivoted QR truncation, as HIP kernels for gfx950.

The package is split so that importing it loads nothing native:

* ``synth``  -- seeded input generators (gates, canonical site pairs, circuits).
  They hold none of the update's arithmetic and serve both the HIP path and
  the oracle used by the tests.
* ``mps``    -- the ctypes binding of ``libmpsgpu.so`` (the C-ABI declared in
  ``include/mps_abi.h``).  Importing it loads the library and fails loudly when
  the library has not been built.
"""

__all__ = ["synth"]
