"""MI355X-native HOTRG hot path (arXiv 2602.05900, Sec. II): the dense
contractions of one coarse-graining step as gfx950 MFMA kernels behind the C
ABI in include/hotrg.h.

Modules: ``binding`` (ctypes binding of libhotrg.so), ``build`` (in-tree
build), ``workloads`` (seeded synthetic inputs), ``accounting`` (FLOP and
byte counts), ``serve`` (continuous-batching solve server).
"""
__all__ = ["binding", "build", "workloads", "accounting"]
