"""MI355X-native FastWalk: random walk centrality from rooted spanning trees sampled by
Wilson's algorithm (Liu, Xie, Zehmakan, Zhang, Section 5), hand-written HIP for gfx950 behind
the C ABI of include/rwc.h.

The HIP library (librwc.so) must be built (``python paper_2510_20604_amd/build.py``); importing
the package raises ImportError if it is missing.  There is no CPU fallback.
"""
from . import _lib

_lib.lib()  # load librwc.so now: fail loudly at import, never later on a silent path

from .api import (Graph, RWCFunction, as_uint64, autotune, autotune_batch, backward, dense_g, estimate,  # noqa: F401,E402
                  estimate_diag, estimate_group, fastchol, prepare_sampling, random_walk_centrality,
                  release_cached_graphs, sample_forests, sample_trap_walks, workspace_status)
from ._lib import RWCError  # noqa: F401,E402
