"""Host-only checks of the request server's admission policy (sk_server_simulate
runs the same Admission code the server uses, with simulated service times)."""
import numpy as np
import pytest

from paper_2606_20195_amd import SketchError, simulate_admission

K = 1024


def test_fifo_slots_and_memory_by_hand():
    a, d = simulate_admission(10 * K, 2, [0, 0, 0, 1], [4 * K, 4 * K, 4 * K, 9 * K], [5, 5, 5, 1])
    assert list(a) == [0, 0, 5, 10] and list(d) == [5, 5, 10, 11]      # slot-bound, then memory-bound
    a, d = simulate_admission(10 * K, 3, [0, 0.5, 1, 1.5], [6 * K, 3 * K, 3 * K, 1 * K], [2, 2, 2, 2])
    assert list(a) == [0, 0.5, 2, 2]                                    # the small request waits its turn


def test_oversized_request_is_refused():
    with pytest.raises(SketchError) as ei:
        simulate_admission(10 * K, 2, [0], [11 * K], [1])
    assert ei.value.code == -6
    with pytest.raises(SketchError):
        simulate_admission(10 * K, 2, [1, 0], [K, K], [1, 1])             # arrivals out of order


@pytest.mark.parametrize("seed", range(6))
def test_invariants_on_random_streams(seed):
    g = np.random.default_rng(seed)
    k = 300
    arrive = np.cumsum(g.exponential(0.005, k))
    fp = g.integers(1, 40, k).astype(np.uint64) * 256 * 1024
    service = g.uniform(0.001, 0.03, k)
    budget, slots = 64 * 256 * 1024, int(g.integers(1, 6))
    a, d = simulate_admission(budget, slots, arrive, fp, service)
    assert np.all(a >= arrive - 1e-15)
    assert np.all(np.diff(a) >= -1e-15)                                   # first come, first admitted
    assert np.allclose(d, a + service)
    events = np.unique(np.concatenate([a, d]))
    for t in events:                                                      # capacity never exceeded
        run = (a <= t) & (d > t)
        assert run.sum() <= slots
        assert fp[run].sum() <= budget
    # admissions happen only at arrivals or completions
    marks = np.concatenate([arrive, d])
    assert all(np.min(np.abs(marks - t)) < 1e-12 for t in a)
