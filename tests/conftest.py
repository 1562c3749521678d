import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(autouse=True)
def _unreached_entries_are_zero(request):
    """In GPU tests, every read of the render statistics also checks that the traversal's
    emission pass reached every interval entry its count pass promised (the library fills
    unreached entries with zero-length ones and counts them; any such entry is a bug)."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    import paper_2310_01881_amd as am
    orig = am.amnerf_render_stats_get

    def checked(ctx):
        st = orig(ctx)
        assert st["n_unreached"] == 0, "traversal emission left %d entries unreached" % st["n_unreached"]
        return st

    am.amnerf_render_stats_get = checked
    try:
        yield
    finally:
        am.amnerf_render_stats_get = orig
