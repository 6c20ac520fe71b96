"""Host test of early termination's cut schedule (paper_0704_2351_amd/csrc/early_cut.h, the outlook of the
paper's conclusion): the header is compiled on its own with g++ into a small driver that feeds it model degree
profiles of the order-c basis of [S; -I] (2s rows whose degrees sum to s (c + 1); the s generator rows grow by
about one every two orders until 2d, then stay at d)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("ecd") / "early_cut_driver")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_0704_2351_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "early_cut_driver.cpp"), "-o", out], check=True)

    def run(L, s, d, step, verify, creep=0):
        lines = subprocess.run([out, str(L), str(s), str(d), str(step), str(verify), str(creep)], check=True,
                               capture_output=True, text=True).stdout.split("\n")
        cuts = [int(x.split()[1]) for x in lines if x.startswith("cut ")]
        end = [x for x in lines if x.startswith("conv ") or x == "none"][0]
        return cuts, (int(end.split()[1]) if end.startswith("conv") else None)

    return run


def test_converges_one_confirming_cut_after_the_stall(driver):
    # generator degree 1500: the rows stall at order 3000; cuts of 512 from L/8 = 625, then one of 128
    cuts, conv = driver(5000, 4, 1500, 512, 128)
    assert cuts == [625, 1137, 1649, 2161, 2673, 3185, 3313]
    assert conv == 3313
    assert 3000 < conv <= 3000 + 512 + 128


@pytest.mark.parametrize("d", [40, 700, 1400])
@pytest.mark.parametrize("s", [1, 8, 16])
def test_never_before_the_stall_and_at_most_a_chunk_after(driver, s, d):
    L, step, verify = 4096 + 1, 512, 128
    cuts, conv = driver(L, s, d, step, verify)
    assert conv is not None and conv >= 2 * d
    assert conv - 2 * d <= max(step, L // 8) + verify
    assert all(b > a for a, b in zip(cuts, cuts[1:])) and cuts[-1] == conv


def test_no_stall_runs_to_full_length(driver):
    # a generator of degree L/2 or more never stalls inside the range: cuts up to L, no convergence
    cuts, conv = driver(5000, 4, 2600, 512, 128)
    assert conv is None and cuts[-1] == 5000


def test_confirming_cuts_double_when_one_row_keeps_growing(driver):
    # row 0 creeps on by one degree every 100 orders after the stall: each confirming cut fails, and their
    # lengths double from 128 up to the chunk length
    cuts, conv = driver(5000, 4, 1500, 512, 128, creep=100)
    assert conv is None
    steps = [b - a for a, b in zip(cuts, cuts[1:])]
    assert steps[:5] == [512] * 5
    assert steps[5:8] == [128, 256, 512]
    assert cuts[-1] == 5000


def test_stall_too_close_to_the_end_is_not_confirmed(driver):
    # the stall at 3800 is seen at the cut 4096, but the confirming cut would pass L = 4097: the range ends
    # (the sequence is complete then) without a confirmation over `verify` orders
    cuts, conv = driver(4097, 8, 1900, 512, 128)
    assert conv is None and cuts[-2:] == [4096, 4097]
