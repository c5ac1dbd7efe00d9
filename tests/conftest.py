import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


def pytest_collection_modifyitems(session, config, items):
    """Run the tests whose child processes make cooperative launches (the
    C-ABI client, the timeline build) before any test of this process makes
    one: while a process that has made a cooperative launch is alive, another
    process's cooperative launch on the same GPU is refused by the runtime."""
    children = ("test_gpu_c_client.py", "test_gpu_timeline.py")
    first = [it for it in items if it.nodeid.split("::")[0].endswith(children)]
    if first:
        rest = [it for it in items if it not in first]
        items[:] = first + rest
