"""Host logic of bench.py: the factorisation schedule it prices the roofline
with is the one the library applies (the tuning table's first matching row,
else the defaults), and its enumeration of trailing-update launches gives
the launch counts the library's profiler reports on the GPU (30 bulk
launches per order-12288 factorisation in four-panel steps down to 4096
rows, 26 down to 2048 rows, 95 next-columns launches in both)."""
import os

import pytest

import bench
from paper_2208_06559_amd import binding as B


def test_schedule_lookup_follows_the_table():
    t = B.load_tuning()
    if t is None:
        pytest.skip("no tuning table committed")
    for n in (900, 3000, 12288, 20000):
        for prec in (B.PREC_FP64, B.PREC_MIXED):
            rows = [r for r in t["schedules"] if r["prec"] == prec and n <= r["n_max"]]
            want = (rows[0]["step_panels"], rows[0]["wide_rows"]) if rows else None
            got = bench.schedule_in_use(t, n, prec)
            if want is not None:
                assert got == want, (n, prec, got, want)


def test_schedule_defaults_without_table(monkeypatch):
    monkeypatch.delenv("BDRPY_STEP_PANELS", raising=False)
    monkeypatch.delenv("BDRPY_WIDE_ROWS", raising=False)
    assert bench.schedule_in_use(None, 12288, B.PREC_MIXED) == (4, 4096)
    monkeypatch.setenv("BDRPY_STEP_PANELS", "2")
    assert bench.schedule_in_use(None, 12288, B.PREC_MIXED)[0] == 2


@pytest.mark.parametrize("sched,bulk", [((4, 4096), 30), ((4, 2048), 26)])
def test_launch_counts_match_the_library(monkeypatch, sched, bulk):
    monkeypatch.delenv("BDRPY_LOOKAHEAD", raising=False)
    assert bench.syrk_per_launch(12288, 4, schedule=sched)[2] == bulk
    assert bench.syrk_per_launch(12288, 4, "next", schedule=sched)[2] == 95
    # every multiply-add of the trailing updates counted once: bulk plus
    # next-columns flops are those of the blocked factorisation's updates
    fl_b, _, nb = bench.syrk_per_launch(12288, 8, schedule=sched)
    fl_n, _, nn = bench.syrk_per_launch(12288, 8, "next", schedule=sched)
    n, nbk = 12288, 128
    want = 0.0
    for k0 in range(0, n, nbk):  # each panel updates the lower triangle below it
        m = n - k0 - nbk
        want += 2.0 * nbk * m * (m + 1) / 2
    assert abs(fl_b * nb + fl_n * nn - want) <= 1e-9 * want
    assert os.path.exists(bench.KERNEL_SOURCE)
