"""Request mix of the serving loop (host side only)."""
import numpy as np

from paper_1208_4772_amd import serving


def test_requests_are_seeded_and_in_range():
    a = serving.make_requests(64, build=False)
    b = serving.make_requests(64, build=False)
    assert [(r.kind, r.K_target, r.P, r.mach, r.steps, r.arrival) for r in a] == \
           [(r.kind, r.K_target, r.P, r.mach, r.steps, r.arrival) for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    # exponential gaps of mean 50 ms: the sample mean of 64 lies within 4 sigma
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 0.05) < 4 * 0.05 / 8
    assert all(2000 <= r.K_target <= 60000 for r in a)
    assert all(500 <= r.steps <= 3000 for r in a)
    assert all(0.3 <= r.mach <= 0.85 for r in a)
    assert {r.P for r in a} == {1, 2, 3, 4, 5}
    assert {r.kind for r in a} == {"cylinder", "airfoil"}


def test_case_sizes_follow_targets():
    reqs = serving.make_requests(6, K_range=(1500, 6000), build=True)
    for r in reqs:
        assert 0.7 * r.K_target <= r.case.K <= 1.3 * r.K_target, (r.kind, r.K_target, r.case.K)
        assert r.case.P == r.P and r.case.steps == r.steps
        assert r.av
