"""MI355X-native vectorised hide-and-seek step (HASE hot path, arxiv 2604.27162).

The HIP library (csrc/) is loaded lazily by paper_2604_27162_amd.hase, so
importing the package (e.g. for the seeded workload generators) loads no
native code.
"""
__version__ = "0.1.0"
