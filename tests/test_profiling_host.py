"""Summaries of kernel traces (no GPU): per-kernel totals and the phase
timeline of multi-task solves, on a small synthetic trace in rocprofv3's
csv layout."""
import csv

import pytest

from paper_1912_13403_amd import profiling

NAMES = ["void (anonymous namespace)::chol_leaf_kernel(int)",
         "void (anonymous namespace)::panel_qr_group_kernel<32>(PanelQrTask const*, int const*)",
         "void (anonymous namespace)::sb2st_group_kernel<32>(Sb2stTask const*, int const*)",
         "void (anonymous namespace)::merge_prep_kernel(int)",
         "void (anonymous namespace)::bt2_group_kernel(Bt2Task const*, int const*)",
         "void (anonymous namespace)::dm_kernel(int)"]


def _trace(path, solves):
    """Two solves 100 ms apart; each: two overlapping leaves (1-5, 2-8 ms),
    the QR group (10-12), two chasing launches (20-30, 31-35), a merge
    (36-40), the stage-2 back-transform (41-50) and D (51-60)."""
    rows = []

    def k(name, a, b):
        rows.append({"Kernel_Name": name, "Start_Timestamp": int(a * 1e6),
                     "End_Timestamp": int(b * 1e6)})
    for base in [100.0 * i for i in range(solves)]:
        k("void at::native::fill_kernel(float)", base, base + 0.1)
        k(NAMES[0], base + 1, base + 5)
        k(NAMES[0], base + 2, base + 8)
        k(NAMES[1], base + 10, base + 12)
        k(NAMES[2], base + 20, base + 30)
        k(NAMES[2], base + 31, base + 35)
        k(NAMES[3], base + 36, base + 40)
        k(NAMES[4], base + 41, base + 50)
        k(NAMES[5], base + 51, base + 60)
    d = path / "trace"
    d.mkdir()
    with open(d / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    return str(d)


def test_stats_totals(tmp_path):
    st = profiling.stats(_trace(tmp_path, 1))
    calls, tot, mean = st["chol_leaf_kernel"]
    assert calls == 2 and tot == pytest.approx(10.0) and mean == pytest.approx(5000.0)
    assert st["sb2st_group_kernel<32>"][0] == 2


def test_timeline_phases(tmp_path):
    out = profiling.timeline(_trace(tmp_path, 2))
    assert len(out) == 2
    for wall, phases in out:
        # the solve runs from the first library kernel (1 ms) to the end of D (60 ms)
        assert wall == pytest.approx(59.0)
        spans = [round(p[2], 6) for p in phases]
        assert spans == [9.0, 10.0, 15.0, 6.0, 9.0, 10.0]
        # device-busy time counts overlapping launches once: leaves 1-8 ms
        assert phases[0][3] == pytest.approx(7.0)
        assert phases[2][3] == pytest.approx(14.0)
        assert phases[0][5][0][0] == "chol_leaf_kernel"
