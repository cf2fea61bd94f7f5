"""MI355X-native Deep Potential (smooth edition) energy / force / virial evaluation.

Importing the package loads nothing native; `paper_2004_11658_amd.dp` loads the HIP
library (`libdp.so`) and fails loudly when it is missing.
"""
__all__ = ["inputs"]
