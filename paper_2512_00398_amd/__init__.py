"""MI355X-native per-DM-trial single-pulse search (HIP for gfx950 behind a C ABI).

``paper_2512_00398_amd.sps`` is the Python binding of ``libsps.so``; build the
library with ``python -m paper_2512_00398_amd.build``.
"""
__all__ = ["sps"]
