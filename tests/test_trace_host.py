"""Host-side decoding of the per-batch trace (Trace.timeline, Trace.levels) on
synthetic records in a CPU buffer: no GPU and no library call."""
import numpy as np
import pytest

import paper_2112_00132_amd as atos

KHZ = 100_000  # 100 MHz record clock: one tick = 10 ns


def _trace(records):
    import torch
    tr = atos.Trace(records=len(records) + 4, device="cpu")
    hdr = np.zeros(8, dtype=np.uint64)
    hdr[0], hdr[1], hdr[2] = len(records), len(records) + 4, KHZ
    raw = np.zeros(len(records), dtype=np.dtype(atos.TRACE_DTYPE))
    for i, rec in enumerate(records):
        raw[i] = rec
    tr.buf[:64] = torch.from_numpy(hdr.view(np.uint8).copy())
    tr.buf[64:64 + 32 * len(records)] = torch.from_numpy(raw.view(np.uint8).copy())
    return tr


def test_timeline_throughput_busy_workers_and_normalisation():
    # two workers: worker 0 busy 0..1000 ticks (10 us) with 2e6 edges; worker 1
    # busy 500..1000 ticks with 1e6 edges; a BSP level record is ignored
    tr = _trace([(0, 1000, 0, 4, 2_000_000, 7), (500, 1000, 1, 2, 1_000_000, 9),
                 (0, 0, 0, atos.TRACE_BSP_LEVEL | 5, 0, 0xFFFFFFFF)])
    tl = tr.timeline(bins=2, useful_edges=1_500_000)
    assert tl["batches"] == 2 and tl["edges"] == 3_000_000
    assert tl["span_ms"] == pytest.approx(0.01)
    # bin 0 (0..5 us): half of worker 0's edges; bin 1: the other half + worker 1's
    assert tl["gteps"] == pytest.approx([1e6 / 5e-6 / 1e9, 2e6 / 5e-6 / 1e9], abs=1e-3)
    assert tl["busy_workers"] == pytest.approx([1.0, 2.0])
    assert tl["overwork"] == pytest.approx(2.0)
    assert tl["gteps_normalised"] == pytest.approx([g / 2 for g in tl["gteps"]], abs=1e-3)
    assert sum(tl["gteps"]) * 5e-6 * 1e9 == pytest.approx(3e6, rel=1e-3)  # edges conserved


def test_levels_of_two_level_synchronous_runs():
    B = atos.TRACE_BSP_LEVEL
    recs = [
        # run 1: levels 0, 1, 2 then its end record (level 3, frontier 0)
        (1000, 0, 0, B | 1, 0, 0xFFFFFFFF), (1300, 0, 1, B | 4, 4, 0xFFFFFFFF),
        (2300, 0, 2, B | 9, 20, 0xFFFFFFFF), (2400, 0, 3, B | 0, 50, 0xFFFFFFFF),
        # a worker batch in between is not a level
        (2500, 2600, 3, 1, 10, 0),
        # run 2: one level and its end; edge counter wrapped past 2^32
        (5000, 0, 0, B | 1, 2 ** 32 - 2, 0xFFFFFFFF), (5100, 0, 1, B | 0, 3, 0xFFFFFFFF),
    ]
    lv = _trace(recs).levels()
    assert lv["level"] == [0, 1, 2, 0]
    assert lv["frontier"] == [1, 4, 9, 1]
    assert lv["edges"] == [4, 16, 30, 5]
    assert lv["us"] == pytest.approx([3.0, 10.0, 1.0, 1.0])
