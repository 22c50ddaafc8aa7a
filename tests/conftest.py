import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


# A planted mistake in a copy of the oracle, for the mutation check of its pins
# (tests/oracle_mutants.py); never set in an ordinary run.
if os.environ.get("WC_ORACLE_MUTANT"):
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle_mutants

    oracle_mutants.install(os.environ["WC_ORACLE_MUTANT"])
