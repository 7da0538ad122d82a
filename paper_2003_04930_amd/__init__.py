"""MI355X-native quantum-PageRank steady-state solver (arXiv:2003.04930).

The compute path is the HIP library ``libqpr.so`` built from ``csrc/``; the
Python binding in :mod:`paper_2003_04930_amd.qpr` only marshals arguments.
Importing the package does not load the library; the first binding call does,
and raises if it is missing.
"""
__all__ = ["inputs"]
