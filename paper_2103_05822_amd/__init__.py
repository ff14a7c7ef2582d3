"""Tucker-compressed FMM far-fields on MI355X (gfx950).

The compute library is ``libtuckfmm.so`` (C ABI in ``include/tuckfmm.h``), built by
:mod:`paper_2103_05822_amd.build`.  :mod:`paper_2103_05822_amd.binding` exposes each
C entry point under the same name; importing the package fails if the library is
missing.
"""
from .binding import *  # noqa: F401,F403
from .binding import FmmError, Layout, exported_symbols  # noqa: F401
