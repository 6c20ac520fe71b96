"""Pins from published values: SplitMix64's first outputs and the iteration
counts of Table "tab:r-time"."""
import os

from oracle import sigma, splitmix

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_splitmix64_known_outputs():
    want = [int(r[0], 16) for r in read_rows("splitmix64_seed0.txt")]
    assert [splitmix.output(0, i) for i in range(3)] == want


def test_splitmix_streams_are_distinct_and_in_range():
    p = 65521
    U = splitmix.block(7, splitmix.STREAM_U, 50, p)
    V = splitmix.block(7, splitmix.STREAM_V, 50, p)
    D = splitmix.block(7, splitmix.STREAM_DROW, 50, p, diag=True)
    assert U != V
    assert all(0 <= x < p for x in U + V)
    assert all(1 <= x < p for x in D)


def test_iteration_counts_of_table_r_time():
    for name, r, it1, itp, procs in read_rows("table_r_time_iterations.txt"):
        r, it1, itp, procs = int(r), int(it1), int(itp), int(procs)
        assert 2 * r + 2 == it1, name
        assert sigma.sequence_length(r, procs) == itp, name
        assert sigma.sequence_length(r, 1) == it1, name
