"""Admission rules of the solve server (paper_2406_00809_amd/csrc/admission.hpp),
compiled with g++ and run on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("adm") / "admission_driver")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-o", exe,
                    os.path.join(HERE, "admission_driver.cpp")], check=True)
    return exe


def plan(driver, budget, used, free_slots, queue, idle, max_skips=8, head_skips=0):
    lines = [f"{budget} {used} {max_skips} {head_skips} {free_slots}",
             f"{len(queue)} " + " ".join(f"{s} {b}" for s, b in queue),
             f"{len(idle)} " + " ".join(f"{s} {b} {t}" for s, b, t in idle)]
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    dec = []
    for ln in out:
        if ln.startswith("END"):
            _, u, hs = ln.split()
            return dec, int(u), int(hs)
        if ln:
            dec.append(ln)
    raise AssertionError(out)


def test_reuse_before_alloc(driver):
    # idle workspace of system 1 is reused; system 2 needs a new one
    dec, used, _ = plan(driver, 100, 30, 4, [(1, 30), (2, 20)], [(1, 30, 5)])
    assert dec == ["REUSE 0 0", "ALLOC 1"]
    assert used == 50


def test_most_recent_idle_reused(driver):
    dec, _, _ = plan(driver, 100, 60, 4, [(1, 30)], [(1, 30, 2), (1, 30, 9)])
    assert dec == ["REUSE 0 1"]


def test_budget_and_lru_eviction(driver):
    # 90 held by idle workspaces of systems 3 (stamp 1), 4 (stamp 7), 5 (stamp 3);
    # a request of 50 bytes needs two evictions, oldest first: 3 then 5
    dec, used, _ = plan(driver, 100, 90, 4, [(1, 50)], [(3, 30, 1), (4, 30, 7), (5, 30, 3)])
    assert dec == ["ALLOC 0 0 2"]
    assert used == 90 - 60 + 50


def test_busy_memory_is_not_evicted(driver):
    # 80 of 100 bytes busy (no idle workspace): a 30-byte request waits
    dec, used, _ = plan(driver, 100, 80, 4, [(1, 30)], [])
    assert dec == [] and used == 80


def test_larger_than_budget_rejected(driver):
    dec, used, _ = plan(driver, 100, 0, 4, [(1, 150), (2, 40)], [])
    assert dec == ["REJECT 0", "ALLOC 1"]
    assert used == 40


def test_slot_limit(driver):
    dec, _, _ = plan(driver, 1000, 0, 2, [(1, 10), (2, 10), (3, 10)], [])
    assert dec == ["ALLOC 0", "ALLOC 1"]


def test_skip_ahead_is_bounded(driver):
    # head (60 bytes) waits for busy memory; small requests may pass it, but
    # only max_skips of them in total while it heads the queue
    q = [(1, 60)] + [(2, 5)] * 6
    dec, used, hs = plan(driver, 100, 50, 16, q, [], max_skips=3)
    assert dec == ["ALLOC 1", "ALLOC 2", "ALLOC 3"]
    assert hs == 3 and used == 65
    # next round, same head still blocked: no further overtaking
    dec, used, hs = plan(driver, 100, 65, 16, [(1, 60)] + [(2, 5)] * 3, [], max_skips=3,
                         head_skips=3)
    assert dec == [] and hs == 3
    # once the head fits it is admitted and the count resets
    dec, used, hs = plan(driver, 100, 40, 16, [(1, 60), (2, 5)], [], max_skips=3, head_skips=3)
    assert dec == ["ALLOC 0"] and hs == 0
