import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")
    # GPU runs check large samples against the oracle in a process pool; fork
    # its workers now, before any test module initialises the GPU
    if "not gpu" not in (config.option.markexpr or ""):
        import oracle_pool
        oracle_pool.start()


def pytest_unconfigure(config):
    import oracle_pool
    oracle_pool.shutdown()
