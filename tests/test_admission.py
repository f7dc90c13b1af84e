"""Host-only tests of the serving daemon's admission control (CPU, no GPU):
the slot, worklist-budget and state-heap bookkeeping of atos_admission.h,
driven through a small C++ harness against a reference model of the same
policy (least used pool with a free slot and room; first-fit heap with
coalescing) and invariants: live allocations never overlap and stay inside
the heap, no pool exceeds its budget, no slot is held twice, and releasing
everything restores one free block and empty pools."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_00132_amd", "csrc")


# the plain build, and the same host code under AddressSanitizer and UBSan
# (any out-of-bounds access, use after free, leak or undefined behaviour in
# the admission bookkeeping aborts the harness and fails the test)
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def harness(request, tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("adm") / f"admission_harness_{request.param}")
    extra = SANITIZE if request.param == "sanitized" else []
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-Wall", *extra, "-I", CSRC, "-o", exe,
                    os.path.join(ROOT, "tests", "admission_harness.cpp")], check=True)
    return exe


class Harness:
    def __init__(self, exe):
        self.p = subprocess.Popen([exe], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)

    def cmd(self, line, lines=1):
        self.p.stdin.write(line + "\n")
        self.p.stdin.flush()
        return [self.p.stdout.readline().strip() for _ in range(lines)]

    def close(self):
        self.p.stdin.close()
        # a sanitizer report (leak, invalid access) at exit makes the status non-zero
        assert self.p.wait(timeout=10) == 0


class Model:
    """The admission policy written out plainly."""

    def __init__(self, slots, pools, cap, base, size):
        self.pools, self.cap = pools, cap
        self.used = [0] * pools
        # free slots per pool as a stack whose top is the lowest slot
        self.slots = [sorted((i for i in range(slots) if i % pools == p), reverse=True)
                      for p in range(pools)]
        self.free = {base: size}

    def admit(self, entries, nbytes):
        pool = None
        for p in range(self.pools):
            if self.slots[p] and self.used[p] + entries <= self.cap and \
                    (pool is None or self.used[p] < self.used[pool]):
                pool = p
        if pool is None:
            return None
        for off in sorted(self.free):
            if self.free[off] >= nbytes:
                rest = self.free.pop(off) - nbytes
                if rest:
                    self.free[off + nbytes] = rest
                break
        else:
            return None
        slot = self.slots[pool].pop()
        self.used[pool] += entries
        return slot, off

    def release(self, slot, entries, off, nbytes):
        self.free[off] = nbytes
        merged = {}
        for o in sorted(self.free):  # coalesce neighbours
            if merged:
                last = max(merged)
                if last + merged[last] == o:
                    merged[last] += self.free[o]
                    continue
            merged[o] = self.free[o]
        self.free = merged
        self.slots[slot % self.pools].append(slot)
        self.used[slot % self.pools] -= entries


@pytest.mark.parametrize("pools", [1, 8])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_admission_matches_model_and_keeps_invariants(harness, pools, seed):
    rng = np.random.default_rng(seed)
    slots, cap, base, size = 32, 1000, 4096, 1 << 20
    h = Harness(harness)
    m = Model(slots, pools, cap, base, size)
    assert h.cmd(f"I {slots} {pools} {cap} {base} {size}") == ["ok"]
    live = {}
    try:
        for step in range(600):
            if live and (rng.random() < 0.45 or len(live) == slots):
                slot = list(live)[int(rng.integers(len(live)))]
                entries, off, nbytes = live.pop(slot)
                assert h.cmd(f"R {slot} {entries} {off} {nbytes}") == ["ok"]
                m.release(slot, entries, off, nbytes)
            else:
                entries = int(rng.integers(1, 400))
                nbytes = int(rng.choice([256, 4096, 65536, 200000]))
                got = h.cmd(f"A {entries} {nbytes}")[0]
                want = m.admit(entries, nbytes)
                if want is None:
                    assert got == "again", (step, got)
                    continue
                assert got == f"ok {want[0]} {want[1]}", (step, got, want)
                slot, off = want
                assert slot not in live
                live[slot] = (entries, off, nbytes)
            # invariants
            spans = sorted((o, o + b) for _, o, b in live.values())
            assert all(a1 <= b0 for (_, a1), (b0, _) in zip(spans, spans[1:]))
            assert all(base <= o and e <= base + size for o, e in spans)
            used = h.cmd("S", 2)[0].split()[1:]
            assert [int(u) for u in used] == m.used
            assert all(int(u) <= cap for u in used)
        for slot, (entries, off, nbytes) in list(live.items()):
            h.cmd(f"R {slot} {entries} {off} {nbytes}")
        used, free = h.cmd("S", 2)
        assert used.split()[1:] == ["0"] * pools
        assert free.split()[1:] == [str(base), str(size)]
    finally:
        h.close()


def test_admission_refuses_what_does_not_fit(harness):
    h = Harness(harness)
    try:
        h.cmd("I 2 1 100 0 1000")
        assert h.cmd("A 101 10") == ["again"]      # over the entry budget
        assert h.cmd("A 10 1001") == ["again"]     # over the heap
        assert h.cmd("A 60 600") == ["ok 0 0"]
        assert h.cmd("A 50 10") == ["again"]       # 60 + 50 entries > 100
        assert h.cmd("A 40 500") == ["again"]      # 600 + 500 bytes > 1000
        assert h.cmd("A 40 400") == ["ok 1 600"]
        assert h.cmd("A 1 1") == ["again"]         # no slot left
        assert h.cmd("R 0 60 0 600") == ["ok"]
        assert h.cmd("A 1 1") == ["ok 0 0"]
    finally:
        h.close()
