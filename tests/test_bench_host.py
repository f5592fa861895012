"""Host logic of the benchmark (no GPU): which steps of the 10k + 20k
protocol are timed, how a stretch is split into graph replays, and the
committed counter summary's guard on the kernel source."""
import itertools

import pytest

import bench


def test_full_protocol_is_timed_in_its_own_proportion():
    p = bench.timed_plan(bench.N_EQUIL + bench.N_SAMPLE - 200, 200, 100)
    assert (p["eq"], p["sa"], p["skip"], p["chunk"]) == (bench.N_EQUIL - 200, bench.N_SAMPLE, 0, 100)


@pytest.mark.parametrize("steps,warmup,chunk", itertools.product((1, 2, 7, 20, 60, 301, 3000, 29800),
                                                                   (0, 5, 200), (0, 2, 7, 100)))
def test_timed_plan_properties(steps, warmup, chunk):
    p = bench.timed_plan(steps, warmup, chunk)
    assert p["eq"] + p["sa"] == steps
    assert 0 <= p["eq"] <= max(0, bench.N_EQUIL - warmup)
    if warmup + steps < bench.N_EQUIL + bench.N_SAMPLE and steps >= 6:
        # short runs time equilibrating and sampling steps about 1 : 2
        assert abs(p["eq"] - steps / 3.0) <= 2.0 or p["eq"] == bench.N_EQUIL - warmup
    if p["sa"] > 0:
        assert warmup + p["eq"] + p["skip"] == max(warmup + p["eq"], bench.N_EQUIL)
    if chunk == 0:
        assert p["chunk"] == 0 and p["chunks"] == []
    else:
        assert p["chunk"] >= 2 and p["chunk"] % 2 == 0
        assert all(c % 2 == 0 and c >= 2 for c in p["chunks"])


class FakeBatch:
    def __init__(self):
        self.calls = []

    def run(self, n, graph_chunk):
        self.calls.append((n, graph_chunk))


@pytest.mark.parametrize("n,chunk", itertools.product((1, 2, 3, 99, 100, 101, 250, 9800), (0, 2, 100)))
def test_advance_covers_every_step_with_even_graphs(n, chunk):
    b = FakeBatch()
    bench.advance(b, n, chunk)
    assert sum(k for k, _ in b.calls) == n
    for k, g in b.calls:
        if g:  # a graph replay runs whole graphs of an even size
            assert g % 2 == 0 and k % g == 0
        else:
            assert chunk == 0 or k == 1


def test_committed_counters_guard_the_kernel_source(tmp_path, monkeypatch):
    # the summary's figures are used only for the kernel it names and while
    # the kernel source still has the hash it records
    import hashlib
    recorded = [line.split(":", 1)[1].strip() for line in open(bench.COUNTERS)
                if line.startswith("source_sha256:")][0]
    current = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    c = bench.committed_counters(bench.FORCE_KERNELS[2])
    if current == recorded:
        assert c is not None and c["traffic"] > 0 and c["flop"] > 0
    else:
        assert c is None
    assert bench.committed_counters("k_force_list<1, 0, 1, 1, 0>") is None
    changed = tmp_path / "md_kernels.hip"
    changed.write_bytes(open(bench.KERNEL_SRC, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(changed))
    assert bench.committed_counters(bench.FORCE_KERNELS[2]) is None
