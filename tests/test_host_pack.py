"""Bin packing of the register-resident kernel (csrc/pack.h), compiled on
its own with g++ and run on the host: the tree-based first fit gives the
packing of the plain first-fit scan, and the balanced capacity keeps every
bin within its limits while spreading small batches over the resident
workgroups."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_15269_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("pack") / "pack_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "pack_driver.cpp"), "-o", exe],
                   check=True)
    return exe


def run(driver, lens, rpw, cap, maxper, slots):
    inp = f"{len(lens)} {rpw} {cap} {maxper} {slots}\n" + \
        " ".join(str(int(x)) for x in lens) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    pos = 0

    def packing():
        nonlocal pos
        nb = int(out[pos])
        pos += 1
        bins = [[int(t) for t in out[pos + k].split()] for k in range(nb)]
        pos += nb
        return bins
    full = packing()
    capb = int(out[pos])
    pos += 1
    return full, capb, packing()


def plain_first_fit(lens, rpw, cap, maxper):
    """First-fit decreasing by a linear scan over the open bins."""
    order = sorted(range(len(lens)), key=lambda i: -lens[i])  # stable
    used, members = [], []
    for i in order:
        pad = -(-lens[i] // rpw) * rpw
        for b in range(len(used)):
            if used[b] + pad <= cap and len(members[b]) < maxper:
                used[b] += pad
                members[b].append(i)
                break
        else:
            used.append(pad)
            members.append([i])
    return members


def check_valid(bins, lens, rpw, cap, maxper):
    seen = sorted(i for b in bins for i in b)
    assert seen == list(range(len(lens)))
    for b in bins:
        assert 1 <= len(b) <= maxper
        assert sum(-(-lens[i] // rpw) * rpw for i in b) <= cap


@pytest.mark.parametrize("seed", range(6))
def test_tree_first_fit_equals_plain_scan(driver, seed):
    rng = np.random.default_rng(seed)
    B = int(rng.integers(1, 400))
    hi = int(rng.choice([16, 40, 256]))
    lens = rng.integers(1, hi + 1, size=B).tolist()
    maxper = int(rng.choice([2, 5, 64]))
    full, _, _ = run(driver, lens, 16, 256, maxper, 10 ** 6)
    assert full == plain_first_fit(lens, 16, 256, maxper)
    check_valid(full, lens, 16, 256, maxper)


def test_balanced_capacity_spreads_small_batches(driver):
    # 512 systems of 16 rows: 32 full bins for 256 resident workgroups
    full, cap, bal = run(driver, [16] * 512, 16, 256, 64, 256)
    assert len(full) == 32 and cap == 32 and len(bal) == 256
    check_valid(bal, [16] * 512, 16, 32, 64)
    # longest system bounds the capacity from below
    lens = [100] * 64
    full, cap, bal = run(driver, lens, 16, 256, 64, 256)
    assert cap == 112 and len(bal) == 64
    check_valid(bal, lens, 16, cap, 64)


@pytest.mark.parametrize("seed", range(4))
def test_balanced_capacity_keeps_the_rounds(driver, seed):
    rng = np.random.default_rng(100 + seed)
    B = int(rng.integers(200, 3000))
    lens = rng.integers(1, int(rng.choice([20, 64, 256])) + 1, size=B).tolist()
    slots = int(rng.choice([64, 256]))
    full, cap, bal = run(driver, lens, 16, 256, 64, slots)
    rounds = -(-len(full) // slots)
    assert len(bal) <= rounds * slots
    assert cap % 16 == 0 and cap <= 256
    assert cap >= max(-(-x // 16) * 16 for x in lens)
    check_valid(bal, lens, 16, cap, 64)
    if cap < 256:  # the capacity one wavefront smaller needs more bins
        smaller = plain_first_fit(lens, 16, cap - 16, 64)
        longest = max(-(-x // 16) * 16 for x in lens)
        assert cap - 16 < longest or len(smaller) > rounds * slots


def test_packing_scales_to_large_batches(driver):
    # 60000 systems: the tree keeps the packing fast (the plain scan would
    # take minutes here)
    import time
    rng = np.random.default_rng(7)
    lens = rng.integers(16, 257, size=60000).tolist()
    t0 = time.perf_counter()
    full, cap, bal = run(driver, lens, 16, 256, 64, 256)
    assert time.perf_counter() - t0 < 20
    check_valid(full, lens, 16, 256, 64)
    check_valid(bal, lens, 16, cap, 64)
