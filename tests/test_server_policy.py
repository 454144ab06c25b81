"""CPU checks of the serving executor's scheduling policy (admission by
memory in arrival order, a first-fit pool, batches of the least remaining
work first, at most two batches in flight), through the library's
virtual-clock simulation, which runs the executor's own policy code without
a device.  Exact timelines are worked out by hand from the policy; random
traces check the invariants."""
import numpy as np
import pytest

def req_bytes(w, h, spp):
    """pool bytes of a request: 8 float32 rays per pixel, then one float32
    radiance per pixel and sample, each part 256-byte aligned"""
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    return up(w * h * 32) + up(w * h * spp * 4)


B64 = req_bytes(64, 64, 1)  # a 64x64 request at 1 spp


@pytest.fixture(scope="module")
def sim():
    from paper_2602_05081_amd import _lib
    return _lib.gf_server_simulate


def test_budget_binds_and_admission_is_fifo(sim):
    # room for the first two 64x64 requests; one tile per batch; 4096 ray-samples per second
    budget = req_bytes(64, 64, 1) + req_bytes(64, 64, 2)
    admit, done, held = sim(budget, 4096, 1, [64] * 3, [64] * 3, [1, 2, 1], [0, 0, 0], [0.0, 0.0, 0.0], 4096.0)
    # t=0: A and B admitted, batches A (ends 1) and B (ends 3); t=1: A done,
    # C admitted, its batch runs after B's (ends 4)
    assert list(admit) == [0.0, 0.0, 1.0]
    assert list(done) == [1.0, 3.0, 4.0]
    assert held == budget


def test_least_remaining_work_first(sim):
    admit, done, _ = sim(1 << 30, 4096, 1, [64, 64], [64, 64], [2, 1], [0, 0], [0.0, 0.0], 4096.0)
    assert list(done) == [3.0, 1.0]
    # multiple scattering counts three times: B (1 spp, multiple) now goes last
    admit, done, _ = sim(1 << 30, 4096, 1, [64, 64], [64, 64], [2, 1], [0, 1], [0.0, 0.0], 4096.0)
    assert list(done) == [2.0, 5.0]


def test_small_late_request_overtakes_remaining_tiles(sim):
    # A: 128x128 = 4 tiles; B (64x64) arrives at 0.5 while two of A's tiles
    # are in flight and takes the next batch
    admit, done, _ = sim(1 << 30, 4096, 1, [128, 64], [128, 64], [1, 1], [0, 0], [0.0, 0.5], 4096.0)
    assert list(admit) == [0.0, 0.5]
    assert list(done) == [5.0, 3.0]


def test_invalid_traces_are_rejected(sim):
    from paper_2602_05081_amd import GfError
    with pytest.raises(GfError):
        sim(B64 - 256, 4096, 4, [64], [64], [1], [0], [0.0], 1.0)  # can never fit
    with pytest.raises(GfError):
        sim(1 << 30, 4096, 4, [64, 64], [64, 64], [1, 1], [0, 0], [1.0, 0.0], 1.0)  # unsorted
    with pytest.raises(GfError):
        sim(1 << 30, 4096, 4, [64], [64], [0], [0], [0.0], 1.0)  # no samples


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_trace_invariants(sim, seed):
    g = np.random.default_rng(seed)
    n = 200
    res = g.choice([128, 256, 512, 1024], size=n)
    spp = g.integers(1, 5, size=n)
    mult = g.integers(0, 2, size=n)
    arrival = np.cumsum(g.exponential(0.05, size=n))
    budget = 3 * 1024 * 1024 * 32
    rate = 2e7
    admit, done, held = sim(budget, 4096, 64, res, res, spp, mult, arrival, rate)
    assert held <= budget
    assert np.all(admit >= arrival) and np.all(done > admit)
    # admission in arrival order
    assert np.all(np.diff(admit) >= 0)
    # the device never runs faster than work_per_s, and is busy from the first arrival
    work = res.astype(float) ** 2 * spp * np.where(mult == 1, 3.0, 1.0)
    assert done.max() >= arrival[0] + work.sum() / rate * (1 - 1e-9)
    # whenever requests wait, the pool could not hold the next one
    for i in np.flatnonzero(admit > arrival):
        assert admit[i] in set(done) or admit[i] in set(arrival)
