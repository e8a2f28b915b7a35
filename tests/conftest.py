import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Test infrastructure: TACCEL_TEST_HOST_LIB names the host build of the library's HIP sources
# (tests/hip_host), which the gpu-marked tests then load through the same C ABI instead of the
# gfx950 build, to run them on a machine without a GPU.  Unset, nothing changes.
HOST_LIB = os.environ.get("TACCEL_TEST_HOST_LIB")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    if HOST_LIB:
        from paper_2504_12908_amd import taccel
        taccel.LIB_PATH = HOST_LIB


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import binding
    if not os.path.exists(binding.LIB_PATH):
        binding.build()
    return binding
