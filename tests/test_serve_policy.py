"""The serving loop's admission and retirement rules on the host, with a
fake executor (tests/serve_policy_sim.cpp over the rules the loop itself
uses, paper_2405_14866_amd/csrc/serve_policy.h): first in first out, the
slot workspace and key capacity, the byte budget of the requests in flight,
solo retries after an overflow, the final capacity error of a request that
overflows alone, retries without sharing after a geometry mismatch, the
batching window, and every request finishing.  A planted fault in the
harness (half of each footprint handed to the rules) must be caught."""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_14866_amd", "csrc")
SIM = os.path.join(ROOT, "tests", "serve_policy_sim.cpp")


def _build(tmp_path, name, *defines):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / name)
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-Werror", *defines, "-I", CSRC, SIM, "-o", exe],
                   check=True, capture_output=True, timeout=120)
    return exe


def _run(exe, *args):
    p = subprocess.run([exe, *[str(a) for a in args]], capture_output=True, text=True, timeout=120)
    return p.returncode, json.loads(p.stdout.strip().splitlines()[-1])


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("sps"), "sps")


# (seed, requests, slots, max_batch, window_us, arrival spacing us)
CASES = [
    (1, 2000, 3, 8, 0, 400),      # sparse arrivals: batches of one
    (5, 2000, 3, 8, 0, 0),        # a burst: full batches against the budget
    (6, 2000, 2, 64, 0, 5),       # large batches, workspace-bound
    (3, 3000, 8, 16, 200, 50),    # batching window
    (4, 500, 1, 1, 0, 0),         # one slot, batches of one
]


@pytest.mark.parametrize("case", CASES)
def test_rules_hold_under_a_fake_executor(sim, case):
    seed, n, slots, max_batch, window, spacing = case
    rc, out = _run(sim, seed, n, slots, max_batch, window, spacing)
    assert out["failures"] == 0, out
    assert rc == 0
    assert out["done"] + out["capacity"] == n
    assert out["capacity"] > 0 and out["retried"] > 0     # oversize requests end in capacity errors
    assert out["max_budget_frac"] <= 1.0
    if spacing == 0 and max_batch > 1:
        assert out["batches_multi"] > 0 and out["overflow_batches"] > out["capacity"]
        assert out["max_budget_frac"] > 0.9                 # the budget, not the queue, bounds admission
    if window > 0:
        assert out["held"] > 0 and out["batches_multi"] > 0


def test_a_planted_budget_fault_is_caught(tmp_path):
    exe = _build(tmp_path, "sps_plant", "-DPLANT_FOOTPRINT")
    rc, out = _run(exe, 5, 2000, 3, 8, 0, 0)
    assert rc != 0 and out["failures"] > 0
    assert out["first_failure"] == "budget accounting"


def test_the_loop_uses_these_rules():
    src = open(os.path.join(CSRC, "serve.hip")).read()
    assert '#include "serve_policy.h"' in src
    for call in ("tg::policy::form_batch(", "tg::policy::retire(", "tg::policy::requeue(", "tg::policy::holds("):
        assert call in src, call
