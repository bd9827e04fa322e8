"""MI355X (gfx950) implementation of the six coupled lattice Boltzmann schemes
of Piredda & Asinari, arXiv:2409.10399, behind the C ABI of include/eelbm.h.

``Lattice`` (binding.py) drives the HIP library ``_lib/libeelbm.so``; build it
with ``python -m paper_2409_10399_amd.build``.
"""
from .binding import (Batch, EelbmError, Lattice, LIB_PATH, lib, map_physical,  # noqa: F401
                      params_from_cfg, state_bytes)
