"""MI355X-native Bloch-simulation hot path (KomaMRI, arXiv 2301.02702).

Importing the package loads nothing native. ``paper_2301_02702_amd.komahip``
binds the HIP library (``libkomahip.so``) and raises if it is missing;
``paper_2301_02702_amd.workloads`` builds seeded synthetic inputs.
"""
__all__ = ["workloads", "komahip"]
