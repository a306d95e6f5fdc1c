"""Compact-triples spin-restricted CCSDT on MI355X.

The compute path is the HIP library ``libcct.so`` built from ``csrc/`` (see
``build.py``); ``binding`` marshals arguments to its C ABI (declared in
``include/cct.h``).  Importing this package does not load the library;
``binding.load()`` does, and raises if it is missing.
"""

__all__ = ["binding"]
