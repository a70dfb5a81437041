"""MI355X-native two-site update of a vectorised density-operator MPO with
Purity-Preserving Truncation (arXiv 2309.08572).

The compute path is libmpdo.so (HIP, gfx950), reached through ``mpdo.MPDO``; PyTorch is
used only for device memory and streams.  ``circuits`` drives the paper-shaped QAOA
circuits through the library.
"""
from .mpdo import MPDO, MPDO_BF16X3, MPDO_FP32, MPDO_FP64, MpdoError, load_library  # noqa: F401
