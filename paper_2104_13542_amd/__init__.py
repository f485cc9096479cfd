"""MI355X-native STORM MPPI step: hand-written HIP kernels behind a C ABI.

The HIP library (``libstorm.so``, built from ``csrc/``) is loaded lazily by
``paper_2104_13542_amd.storm``; importing this package alone loads nothing, so
the seeded input module ``paper_2104_13542_amd.inputs`` can be used without a GPU.
"""
__version__ = "0.1.0"
