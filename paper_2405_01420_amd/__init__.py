"""MI355X-native short-range nonbonded forces (grid sort, cluster-pair list, LJ + Ewald
real-space kernel) behind a C-ABI library.  Submodules load the compiled library lazily."""
__all__ = ["synth"]
