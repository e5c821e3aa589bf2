"""Hierarchical Particle-Mesh (arXiv:1906.10734) for AMD MI355X.

The method is implemented in the HIP library ``libhpm.so`` (C ABI: include/hpm.h); the module
``paper_1906_10734_amd.hpm`` is its Python binding. Build the library with
``python -m paper_1906_10734_amd.build``.
"""
