"""MI355X-native conservative dG Arakawa right-hand side.

The compute path is the HIP library ``libdgark.so`` built from ``csrc/``;
``paper_1311_7477_amd.dg`` is its thin ctypes binding.  Importing this
package loads nothing: the library is opened on first use and its absence
raises an error (there is no fallback path).
"""
__all__ = ["dg", "inputs"]
