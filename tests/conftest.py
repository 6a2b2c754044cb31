import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _library_built_from_this_tree(request):
    """GPU sessions run the library built from the sources in this tree: a
    stale build fails here instead of passing on old kernels."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        from paper_2303_02210_amd import _ffi, build
        got, want = _ffi.built_source_hash(), build.source_hash()
        assert got == want, f"liblbmgrow.so was built from sources {got}, the tree is {want}"
        print(f"\n{_ffi.lib().lbm_version().decode()}", flush=True)
