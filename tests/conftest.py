import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")
    # Load what is built; build only what is missing (the oracle and librfp.so).
    from oracle import build as obuild
    if not os.path.exists(obuild.LIB):
        obuild.build()
    from paper_0901_1696_amd import build as rbuild
    if not os.path.exists(rbuild.LIB):
        rbuild.build()
