"""Host-side logic of the serving loop: admission order, percentiles and the
arrival process (no GPU needed)."""
import math

from paper_2008_01765_amd import serving


def test_admit_prefix_is_first_come_first_served():
    assert serving.admit_prefix([], 10) == 0
    assert serving.admit_prefix([3, 3, 3], 10) == 3
    assert serving.admit_prefix([3, 3, 3, 3], 10) == 3
    # a large head blocks smaller requests behind it
    assert serving.admit_prefix([11, 1, 1], 10) == 0
    assert serving.admit_prefix([0, 0, 5, 6], 10) == 3
    assert serving.admit_prefix([10], 10) == 1


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serving.percentile(v, 50) == 50
    assert serving.percentile(v, 99) == 99
    assert serving.percentile(v, 100) == 100
    assert serving.percentile(v, 0) == 1
    assert serving.percentile([7.0], 99) == 7.0
    assert serving.percentile([3, 1, 2], 50) == 2


def test_poisson_arrivals_rate_and_order():
    a = serving.poisson_arrivals(20000, rate_per_s=500.0, seed=9)
    assert all(x < y for x, y in zip(a, a[1:]))
    gaps = [a[0]] + [y - x for x, y in zip(a, a[1:])]
    mean = sum(gaps) / len(gaps)
    # exponential gaps: mean 1/rate, standard error 1/(rate sqrt(N))
    assert abs(mean - 1 / 500.0) < 5 * (1 / 500.0) / math.sqrt(len(gaps))
    # memorylessness check: fraction of gaps above the mean is e^-1
    frac = sum(g > 1 / 500.0 for g in gaps) / len(gaps)
    assert abs(frac - math.exp(-1)) < 0.02
    assert serving.poisson_arrivals(5, 10.0, seed=1) == serving.poisson_arrivals(5, 10.0, seed=1)
