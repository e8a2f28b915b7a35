"""The gpu-marked test files run against the host build of the library's HIP sources
(tests/hip_host: guard-page allocations, every lane a fiber, the blocks of a launch on several
host threads), through the same C ABI, on a machine without a GPU.

Hours of CPU time for the whole set, so it runs only when asked for:

    TACCEL_HOST_SUITE=1 python -m pytest tests/test_host_gpu_suite.py -q

or one file at a time with TACCEL_HOST_SUITE_FILES="tests/test_gpu_parity.py ...".  Each file
runs in a child pytest with TACCEL_TEST_HOST_LIB pointing at the host build; a memory error
ends that child with the faulting allocation named on stderr.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FILES = os.environ.get("TACCEL_HOST_SUITE_FILES", "").split() or sorted(
    os.path.join("tests", f) for f in os.listdir(HERE) if f.startswith("test_gpu") and f.endswith(".py"))

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("TACCEL_HOST_SUITE") != "1",
                                 reason="set TACCEL_HOST_SUITE=1 to run the gpu tests on the host build")]


@pytest.fixture(scope="module")
def host_lib():
    sys.path.insert(0, os.path.join(HERE, "hip_host"))
    try:
        import build as hb
    finally:
        sys.path.pop(0)
    return hb.build()


@pytest.mark.parametrize("path", FILES)
def test_gpu_file_on_host_build(host_lib, path):
    env = dict(os.environ, TACCEL_TEST_HOST_LIB=host_lib)
    p = subprocess.run([sys.executable, "-u", "-m", "pytest", path, "-m", "gpu", "-q", "-x", "-rs",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True)
    sys.stdout.write(p.stdout[-4000:])
    assert p.returncode in (0, 5), (p.returncode, p.stdout[-4000:], p.stderr[-4000:])
