"""Plain FP64 CPU oracle for the conservative dG Arakawa scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library; it builds every operator itself
from the paper's definitions (Einkemmer & Wiesenberger, "A conservative
discontinuous Galerkin scheme for the 2D incompressible Navier-Stokes
equations", Sections 2-6).
"""
from .dg_oracle import *  # noqa: F401,F403
