"""MI355X (gfx950) LeanVec search: Python binding of the C-ABI library liblv.so.

The hot path (query projection on the matrix cores, LVQ-scored best-first
graph traversal, float16 re-ranking) runs in hand-written HIP kernels; this
package only marshals arguments (see ``_lib``).  Build with
``python paper_2312_16335_amd/build.py``.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import Index, LVError, exported_names, load  # noqa: F401
