"""Photo-SLAM photorealistic-mapping hot path on AMD MI355X (gfx950).

``gs`` binds the C interface of libgs (include/gs.h); ``mapper`` chains its
calls into a mapping iteration.  Importing ``gs`` requires the built
``libgs.so`` (``paper_2311_16728_amd.build.build()``).
"""

__all__ = ["gs", "mapper", "build"]
