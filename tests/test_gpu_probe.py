"""The memory-roof probes (lidar_probe_stream / lidar_probe_gather) run, read only, and stay in bounds.

They measure, they compute nothing of the simulation: the checks are that every launch succeeds, that the
sink is never written (the data never sums to the improbable value) and that a gather over a table of one
128-byte line, whose every index is line 0, behaves like any other size.
"""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


@pytest.mark.parametrize("n_words", [4, 4 * 1000 + 4, 1 << 22])
def test_stream_probe(L, n_words):
    buf = torch.randint(-2**31, 2**31 - 1, (n_words,), dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    run = L.probe_stream_launcher(buf, sink)
    for _ in range(3):
        assert run() == 0
    torch.cuda.synchronize()
    assert sink.item() == 0.0


@pytest.mark.parametrize("lines", [1, 3, 12345])
@pytest.mark.parametrize("chase", [False, True])
def test_gather_probe(L, lines, chase):
    table = torch.randint(-2**31, 2**31 - 1, (lines * 32,), dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    run = L.probe_gather_launcher(table, 64, 16, chase, sink)
    for _ in range(3):
        assert run() == 0
    torch.cuda.synchronize()
    assert sink.item() == 0.0
