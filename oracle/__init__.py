"""CPU oracle for particle data binning: test infrastructure only.

Callers: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``.  Nothing in the product package imports this package.
"""
from . import binning_oracle  # noqa: F401
