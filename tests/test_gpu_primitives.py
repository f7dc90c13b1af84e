"""GPU checks of the primitives the worklist relies on (through the C-ABI).

The worklist publishes a task by completing the stores of its data (a wait on
the wavefront's outstanding memory operations) before the store of the slot
word, and every shared location is read with agent-scope loads; no L2-wide
release/acquire fences are used.  The message-passing litmus test checks
that pattern across XCDs: a reader that sees the flag must see the data.
"""
import pytest

pytestmark = pytest.mark.gpu


def _atos():
    import paper_2112_00132_amd as atos
    return atos


@pytest.mark.parametrize("pairs,rounds", [(100, 20000), (512, 2000)])
def test_message_passing_litmus_sees_no_stale_data(pairs, rounds):
    import torch
    atos = _atos()
    buf = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    ms = atos.microbench("litmus_mp", buf, iters=rounds, grid=2 * pairs, block=64)
    stale, giveups, completed = buf[:3].cpu().tolist()
    assert ms > 0
    assert giveups == 0, "a bounded spin gave up (pair not co-resident?)"
    assert completed == pairs * rounds
    assert stale == 0


@pytest.mark.parametrize("kind", ["copy", "atomic_add_f32", "atomic_add_f64", "atomic_min_u32",
                                  "gather_plain", "gather_coherent"])
def test_microbench_kinds_run(kind):
    import torch
    atos = _atos()
    buf = torch.zeros(1 << 22, dtype=torch.int32, device="cuda")
    ms = atos.microbench(kind, buf, iters=1 << 20, grid=1024, block=256)
    assert ms > 0


def test_microbench_rejects_bad_arguments():
    import torch
    atos = _atos()
    buf = torch.zeros(1 << 12, dtype=torch.int32, device="cuda")
    with pytest.raises(atos.AtosError):
        atos.microbench("copy", buf, iters=1, grid=1, block=100)  # not a multiple of 64
    with pytest.raises(atos.AtosError):
        atos.microbench("litmus_mp", buf, iters=10, grid=1000, block=64)  # buffer too small


def test_device_clock_rate_matches_the_reported_rate():
    """The worklist deadlines count the constant-rate device clock at 100 MHz;
    check that rate against HIP event time."""
    import torch
    atos = _atos()
    buf = torch.zeros(1 << 12, dtype=torch.int64, device="cuda")
    ticks = 20_000_000  # 0.2 s at 100 MHz
    ms = atos.microbench("clock", buf, iters=ticks, grid=1, block=64)
    t0, t1, spins = buf[:3].cpu().tolist()
    assert spins < (1 << 26), "the clock did not advance"
    rate_khz = (t1 - t0) / ms
    print("device clock", rate_khz, "kHz over", ms, "ms,", spins, "reads")
    assert 0.8 * 100000 < rate_khz < 1.25 * 100000
