"""The serving pool's admission policy on the CPU (host code only): memory budget, slots and the
resident-node cap, first come first served, and a request whose memory the device refuses; and
how a step call is split into graph replays and direct launches.  Compiles tests/pool_policy_check.cpp against the
policy header with g++ and checks which requests are resident after each event."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lines():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "policy")
        subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror",
                        "-I", os.path.join(ROOT, "paper_1812_05401_amd", "csrc"),
                        os.path.join(ROOT, "tests", "pool_policy_check.cpp"), "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {ln.split()[0]: ln.split()[1:] for ln in out.splitlines()}


def test_refused_memory_waits_while_resident_and_fails_when_alone(lines):
    assert lines["refused"] == ["[0]", "[2]failed:1"]


def test_step_chunks_add_up_and_fit_an_int(lines):
    """vplbm_step's split of a call: graph replays while a whole replay remains, then direct
    enqueues of at most 2^30 steps (their launch offsets are ints), adding up to the call."""
    assert lines["plan_short"] == ["0", "3", "ok"]
    assert lines["plan_graph"] == ["2", "44", "ok"]
    assert lines["plan_nograph"] == ["0", "1001", "ok"]
    assert lines["plan_2e31"] == ["0", str(1 << 30), str(1 << 30), "5", "ok"]
    assert lines["plan_2e32_graph"][0] == str(((1 << 32) + 7) // 128)
    assert lines["plan_2e32_graph"][1:] == [str(((1 << 32) + 7) % 128), "ok"]


def test_budget_binds_and_the_head_blocks(lines):
    assert lines["budget"] == ["[0]", "[1,2]"]


def test_slots_bind(lines):
    assert lines["slots"] == ["[0,1]", "[0,2]"]


def test_node_cap_binds_while_something_is_resident(lines):
    assert lines["cap"] == ["[0]", "[1,2]"]


def test_a_request_larger_than_the_cap_runs_alone(lines):
    assert lines["oversized"] == ["[0]", "[1]"]


def test_no_cap(lines):
    assert lines["nocap"] == ["[0,1,2]"]
