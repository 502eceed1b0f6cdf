"""MI355X-native PBD-R rigid-body solver substep (arXiv 2603.14634).

The solver is the HIP library ``libpbdr.so`` behind the C ABI in
``include/pbdr.h``; ``binding`` marshals arguments to it and ``scenes`` makes
seeded synthetic inputs.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "binding"]
