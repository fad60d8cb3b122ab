"""Host-side accounting of bench.py: which blocks of a dense load run on the
dense kernels (the library's default placement rule) and the algorithmic
bytes and flops of an iteration that the roofline is priced with."""
import importlib.util
import os

import numpy as np

import workloads

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench", os.path.join(_ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_block_placement_follows_the_default_rule():
    # 64-row, 1024-column blocks of a 90%-observed matrix: all dense
    wl = workloads.dense_tweedie(I=256, J=4096, B=4, name="t")
    dense, cnt, rows, cols = bench.block_placement(wl)
    assert dense.all() and cnt.sum() == wl.nnz
    assert list(rows) == [64] * 4 and list(cols) == [1024] * 4
    # 128-column blocks: narrower than 256 columns, all as coordinates
    wl = workloads.dense_tweedie(I=256, J=4096, B=32, name="t")
    assert not bench.block_placement(wl)[0].any()
    # the 256 x 256 Poisson test case (64-column blocks): coordinates
    assert not bench.block_placement(workloads.dense_poisson())[0].any()


def test_block_placement_density_and_height_limits():
    wl = workloads.dense_tweedie(I=260, J=1024, B=2, name="t")    # 130-row blocks
    assert not bench.block_placement(wl)[0].any()
    wl = workloads.dense_tweedie(I=256, J=1024, B=2, heldout=0.75, name="t")   # 25% observed
    assert not bench.block_placement(wl)[0].any()


def test_algorithmic_cost_counts_cells_entries_and_extras():
    wl = workloads.dense_tweedie(I=256, J=4096, B=4, name="t")
    wl.burn_in, wl.thin = 10, 5
    dense, cnt, rows, cols = bench.block_placement(wl)
    cells, entries = bench.part_work(wl, dense, cnt, rows, cols)
    assert list(cells) == [256 * 4096 // 4] * 4 and not entries.any()
    ho_p = np.array([7, 0, 0, 0])
    factors = 8 * (wl.I + wl.J) * wl.K
    assert bench.algorithmic_cost(wl, cells, entries, ho_p, 0, 0) == (4.125 * cells[0] + factors, 6 * wl.K * cells[0])
    kept = bench.algorithmic_cost(wl, cells, entries, ho_p, 15, 0)[0]
    assert kept == 4.125 * cells[0] + factors + 16 * 7 + 32 * (wl.I + wl.J) * wl.K
    assert bench.algorithmic_cost(wl, cells, entries, ho_p, 16, 0)[0] == 4.125 * cells[0] + factors + 16 * 7
    # values stored in BF16: 2 bytes and the training bit per cell
    assert bench.algorithmic_cost(wl, cells, entries, ho_p, 0, 0, bench.VALUE_BYTES["bf16v"])[0] == \
        2.125 * cells[0] + factors
    assert bench.VALUE_BYTES["f32"] == bench.VALUE_BYTES["bf16"] == 4
    # the same matrix in 128-column blocks: every training entry as coordinates
    wl = workloads.dense_tweedie(I=256, J=4096, B=32, name="t")
    dense, cnt, rows, cols = bench.block_placement(wl)
    cells, entries = bench.part_work(wl, dense, cnt, rows, cols)
    assert not cells.any() and entries.sum() == wl.nnz
    assert bench.algorithmic_cost(wl, cells, entries, np.zeros(32, int), 0, 3) == (
        8 * entries[3] + 8 * (wl.I + wl.J) * wl.K, 0)


def test_traffic_copy_reference_reproduces_the_copy():
    """The stored copy reference scales its own counters back to the bytes the
    copy moves (256 MiB read, 256 MiB written), and every stored run is priced
    with it: read and write bytes both positive, the read scale between the
    64- and 128-byte request sizes FETCH_SIZE can mistake."""
    import json
    with open(os.path.join(_ROOT, "profiles", "traffic.json")) as f:
        data = json.load(f)
    ref = data["copy_reference"]
    assert abs(ref["FETCH_SIZE_KiB"] * ref["fetch_scale"] - 262144.0) < 1.0
    assert abs(ref["WRITE_SIZE_KiB"] * ref["write_scale"] - 262144.0) < 1.0
    assert 1.0 <= ref["fetch_scale"] <= 2.0 + 1e-3
    for key, run in data["runs"].items():
        kind = "dense" if key.startswith("dense") else "sparse"
        want = 1024.0 * (run["FETCH_SIZE_KiB"] * ref["fetch_scale"] + run["WRITE_SIZE_KiB"] * ref["write_scale"])
        got = bench.measured_traffic(key, kind)
        assert got is None or abs(got - want) < 1.0
