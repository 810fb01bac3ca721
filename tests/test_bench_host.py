"""Host logic of bench.py (no GPU): algorithmic bytes, visit counts, the CPU baseline's
sample, the counter summaries it reads, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bytes_per_update_of_the_medium_workload():
    # 12-byte entry + 2 x 400 B for w_i + 2 x 400 B per (worker, item) visit: with every one
    # of 17,770 items visiting all 256 workers, 2 x 400 x 4,549,120 / 98.6 M
    assert bench.bytes_per_update(100, 4, 4, 17_770 * 256, 98_600_000) == pytest.approx(848.91, abs=0.01)
    # BF16 w_i halves the row term only
    assert bench.bytes_per_update(100, 2, 4, 17_770 * 256, 98_600_000) == pytest.approx(448.91, abs=0.01)


def test_visits_per_epoch_counts_worker_item_pairs():
    import torch

    row = torch.tensor([0, 1, 2, 3, 4, 5, 5], dtype=torch.int32)
    col = torch.tensor([0, 0, 1, 1, 1, 2, 0], dtype=torch.int32)
    # workers own rows [0,2), [2,4), [4,6): pairs (0,0) (1,1) (2,1) (2,2) (2,0)
    assert bench.visits_per_epoch(row, col, 3, [0, 2, 4, 6]) == 5


@pytest.mark.parametrize("sched", ["perm", "uniform", "ring"])
def test_counter_summaries_are_used_only_for_their_kernel_source(sched):
    """A counter summary names the kernel source it was taken at; bench.py reports its
    traffic only while the source is unchanged (else `traffic` is null)."""
    kernel = bench.KERNELS[sched]
    path = bench.counters_path(kernel, sched)
    assert os.path.exists(path), path
    kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    traffic = bench.measured_traffic(kernel, sched)
    if kv["kernel_source_sha256"] != bench.kernel_source_hash():
        assert traffic is None
        return
    assert traffic is not None
    # the summary's per-update figure is the same bytes over the workload's ratings
    assert traffic / 98_600_000 == pytest.approx(float(kv["hbm_bytes_per_update"]), rel=2e-3)


def test_stale_counter_summary_is_not_used(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("k_worker_async", "perm") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_visits_per_epoch_in_chunks_matches_one_pass():
    import torch

    g = torch.Generator().manual_seed(3)
    row = torch.randint(0, 500, (20_000,), generator=g, dtype=torch.int32)
    col = torch.randint(0, 90, (20_000,), generator=g, dtype=torch.int32)
    rs = [0, 70, 200, 330, 500]
    q = torch.searchsorted(torch.tensor(rs), row.long(), right=True) - 1
    expect = int(torch.unique(q * 90 + col.long()).numel())
    assert bench.visits_per_epoch(row, col, 90, rs) == expect
    assert bench.visits_per_epoch(row, col, 90, rs, chunk=777) == expect


def test_block_sample_keeps_the_leading_block_in_order():
    import numpy as np

    import synth

    p = synth.small_case(300, 120, 6_000, seed=9, degrees="zipf")
    m_s, n_s, r, c, v = bench.block_sample(p, 0.5, 0.25, chunk=1_000)
    assert (m_s, n_s) == (150, 30)
    row, col, val = p.row.numpy(), p.col.numpy(), p.val.numpy()
    sel = (row < 150) & (col < 30)
    assert np.array_equal(r, row[sel]) and np.array_equal(c, col[sel]) and np.array_equal(v, val[sel])
    assert r.size > 0
