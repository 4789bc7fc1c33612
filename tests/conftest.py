import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The planted-mistake check runs the oracle's pins against a modified copy
# of the oracle package kept in this directory.
if os.environ.get("ORACLE_PACKAGE_DIR"):
    sys.path.insert(0, os.environ["ORACLE_PACKAGE_DIR"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")
