"""MI355X-native hierarchical interpolative factorization (HIF) of the 3-D
7-point elliptic operator: C-ABI HIP library (libhif.so) plus a thin binding.

Import `paper_1607_00346_amd.hif` for the binding; this package init loads
nothing so that building and CPU-only tooling work without a GPU.
"""
