import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")


def _ensure_built():
    """Build the small CPU-side libraries if they are absent (gcc, a second or two).
    The HIP library is never built here: __graft_entry__.build() does that."""
    import oracle.build
    import synth.build
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build.build()


_ensure_built()


@pytest.fixture(scope="session")
def c1_graph():
    """Scale-12 R-MAT graph, 2^16 edges, weights 1..100 (seeds 1 and 2)."""
    import synth
    g = synth.rmat_csr(12, 1 << 16)
    w = synth.weights(g.m)
    return g, w
