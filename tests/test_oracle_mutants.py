"""Mutation check of the oracle's pins: every planted mistake listed in
tests/oracle_mutants.py must make at least one pin fail.  Each mutant runs
the pin files in a fresh process (-x: it stops at the first failure) with
WC_ORACLE_MUTANT naming the mutant; exit status 1 means that tests ran and
one failed.  0 would mean the mutant survived every pin; any other status
means the run did not get as far as the tests (for instance a mutation site
that no longer matches the oracle's text)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)

import oracle_mutants  # noqa: E402

PIN_FILES = ["test_oracle_pins.py", "test_readings.py", "test_oracle_grad.py"]


def run_pins(name):
    env = dict(os.environ, WC_ORACLE_MUTANT=name, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + [os.path.join(HERE, f) for f in PIN_FILES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = [line for line in r.stdout.splitlines() if line.startswith("FAILED")]
    return name, r.returncode, failed[:1], r.stdout[-400:] + r.stderr[-400:]


def test_mutation_sites_match_the_oracle():
    for name, (kind, find, repl) in oracle_mutants.MUTANTS.items():
        assert oracle_mutants.patched(kind, find, repl) is not None, name


@pytest.mark.timeout(900)
def test_every_planted_mistake_fails_a_pin():
    with ThreadPoolExecutor(max_workers=4) as pool:
        results = list(pool.map(run_pins, sorted(oracle_mutants.MUTANTS)))
    for name, rc, failed, _ in results:
        print(name, rc, failed)
    survivors = [name for name, rc, _, _ in results if rc == 0]
    broken = [(name, rc, tail) for name, rc, _, tail in results if rc not in (0, 1)]
    assert not survivors, survivors
    assert not broken, broken
