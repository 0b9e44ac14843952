"""MI355X-native delta-stepping single-source shortest paths.

The compute path is libsssp.so (hand-written HIP for gfx950) behind the C ABI
in include/sssp.h; ``paper_1911_06895_amd.sssp`` is its Python binding and
``paper_1911_06895_amd.graphs`` holds the seeded input generators.
"""
from . import graphs  # noqa: F401  (numpy only)

__all__ = ["graphs", "sssp", "build"]
