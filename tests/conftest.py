import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--fwi-lib", default=None,
                     help="load this build of libfwi_mi355x.so (e.g. the sanitizer build)")
    parser.addoption("--oracle-lib", default=None,
                     help="load this build of the oracle (e.g. the sanitizer build)")


def pytest_configure(config):
    lib = config.getoption("--fwi-lib")
    if lib:
        try:  # torch's HIP runtime must be the one the library binds to
            import torch  # noqa: F401
        except ImportError:
            pass
        from paper_2507_10804_amd import fwi
        fwi.load_library(os.path.abspath(lib))
    olib = config.getoption("--oracle-lib")
    if olib:
        import oracle
        oracle.use_library(os.path.abspath(olib))
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU-only test")
