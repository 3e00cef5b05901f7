"""Wall-function bounce (WFB) LBM-LES channel step on AMD MI355X (gfx950).

Han, Ooka & Kikumoto, "A wall function approach in lattice Boltzmann method:
algorithm and validation using turbulent channel flow" (arXiv 2009.04352).
The computation lives in liblbmwf.so (HIP kernels behind the C ABI of
include/lbmwf.h); this package only marshals arguments and provides device
memory and streams through PyTorch.
"""
from ._lib import LbmError, lib  # noqa: F401
from .channel import (BOUNDARIES, STORES, Batch, Channel, codec_roundtrip, copy_probe, device_wall_utau,  # noqa: F401
                      spalding_uplus)
