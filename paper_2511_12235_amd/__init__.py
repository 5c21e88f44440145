"""Exact cone-beam system matrix (arXiv 2511.12235) on MI355X.

``projector.SystemMatrix`` applies W and W^T through the HIP library
(``libsm.so``, C ABI in include/sm.h); ``workloads`` describes scans and
seeded synthetic inputs.  Submodules are imported on demand so that the
input generators stay usable without a GPU.
"""
__all__ = ["projector", "workloads", "serve", "experiments"]
