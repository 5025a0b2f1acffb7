"""MI355X-native finite-element lattice Boltzmann for binary fluids.

Importing the package loads nothing native; `paper_1608_01906_amd.felbm`
is the binding of the HIP library and fails loudly if it is not built.
"""
__all__ = ["inputs", "felbm"]
