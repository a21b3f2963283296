"""Host logic of the benchmark script (no GPU): the streaming batch schedule
and the flop count the roofline line is computed from."""

import math

import bench


def test_ramp_batches_cover_every_pulse_in_order():
    for n, first, factor in [(1000, 16, 4), (100, 5, 4), (1, 5, 4), (7, 1, 2), (64, 64, 4)]:
        b = bench.ramp_batches(n, first, factor)
        assert sum(b) == n and min(b) >= 1
        assert b[0] == min(first, n)
        # each batch is `factor` times the one before, except the last (the remainder)
        for prev, cur in zip(b[:-2], b[1:-1]):
            assert cur == prev * factor
        assert len(b) == 1 or b[-1] <= b[-2] * factor


def test_ramp_batches_of_the_benchmark():
    assert bench.ramp_batches(1000, 16, 4) == [16, 64, 256, 664]
    assert bench.ramp_batches(100, 5, 4) == [5, 20, 75]


def test_roofline_flop_count_is_the_nominal_count():
    # 5 N log2 N + 2 N + 2 L per pulse-gate spectrum at N = 16384, L = 1000
    n, L = 16384, 1000
    want = 5 * n * math.log2(n) + 2 * n + 2 * L
    assert want == 1_181_648
    assert bench.flops_per_spectrum(n, L) == want
