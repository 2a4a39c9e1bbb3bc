"""DiskChunGS mapping-step hot path on MI355X (gfx950).

``dcgs`` is the ctypes binding of libdcgs (C ABI in ``include/dcgs.h``);
``mapping`` sequences its calls into one mapping iteration; ``render``
wraps forward/backward as a ``torch.autograd.Function``.  Build the library
with ``python -m paper_2511_23030_amd.build``.
"""
from . import dcgs  # noqa: F401

__all__ = ["dcgs"]
