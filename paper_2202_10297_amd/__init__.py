"""pvjp: tape-free reverse-mode (VJP) rules for bulk-parallel operators on MI355X.

The compute path is the HIP library ``libpvjp.so`` (C ABI declared in
``include/pvjp.h``).  ``capi`` binds it through ctypes under the same names;
``ops`` marshals torch tensors (device memory and streams only) into those
calls.  Importing this package loads nothing; the library is loaded on first
use and its absence is an error, never a fallback.
"""

__all__ = ["capi", "ops", "workloads"]
