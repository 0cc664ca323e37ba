import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")


def _ensure_built():
    """Build whichever library is absent (never rebuilds one that exists:
    __graft_entry__.build() is the step that recompiles everything)."""
    import oracle.build
    import synth.build
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build.build()
    if not os.path.exists(os.path.join(ROOT, "paper_1606_08150_amd", "libwc.so")):
        import paper_1606_08150_amd.build
        paper_1606_08150_amd.build.build()


_ensure_built()


@pytest.fixture(scope="session")
def c1_graph():
    """Scale-12 R-MAT graph, 2^16 edges, weights 1..100 (seeds 1 and 2)."""
    import synth
    g = synth.rmat_csr(12, 1 << 16)
    w = synth.weights(g.m)
    return g, w


@pytest.fixture(scope="session")
def ctx():
    """One libwc context on cuda:0 for the whole GPU session."""
    import torch
    from paper_1606_08150_amd import wc
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    c = wc.Context(0)
    yield c
    c.close()
