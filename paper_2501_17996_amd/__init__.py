"""MI355X-native PDMCF solver: PDHG for destination-aggregated all-pairs
multicommodity network flow (Zhang & Boyd, arXiv 2501.17996).

The solver is the C-ABI library ``libmcf.so`` (HIP kernels for gfx950); the
Python binding in ``mcf.py`` only marshals arguments.  Nothing is imported
eagerly so that ``instances`` can be used on machines without a GPU.
"""
__all__ = ["instances", "mcf"]
