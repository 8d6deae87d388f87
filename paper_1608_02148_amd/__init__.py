"""MI355X (gfx950) randomized SVD / PCA: Erichson et al., arXiv:1608.02148.

The computation lives in ``librsvd_mi355x.so`` (hand-written HIP, C ABI in
``include/rsvd_mi355x.h``); this package only binds it for torch tensors.
"""
from .api import rsvd, rpca, handle, sync_info, new_info  # noqa: F401
