"""MI355X-native multigrid hierarchical data refactoring.

``libmgr.so`` (HIP, gfx950) implements the decomposition and recomposition of
Chen et al., arXiv 2105.12764, behind the C ABI in ``include/mgr.h``;
:mod:`paper_2105_12764_amd.mgr` is its Python binding.  Importing this package
loads nothing; the library is loaded on first use.
"""

__all__ = ["mgr", "synth", "build"]
