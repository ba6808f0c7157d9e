"""Pins of the oracle's lane tracker (alpha-beta filter on each lane's start column, greedy
gated association): the first steps worked by hand, the zero steady-state error of an
alpha-beta filter on a constant-rate ramp, its noise-variance reduction against the published
closed form, gating, births and deaths, the association order and the capacity."""
import numpy as np

import oracle


def test_first_steps_by_hand():
    s = oracle.TrackState()
    oracle.track_update(s, [100])
    assert s.n == 1 and s.id[0] == 0 and s.x[0] == 100.0 and s.dx[0] == 0.0 and s.hits[0] == 1
    oracle.track_update(s, [104])            # x_hat 100, r 4: x 102, dx 0.4
    assert abs(s.x[0] - 102.0) < 1e-12 and abs(s.dx[0] - 0.4) < 1e-12 and s.hits[0] == 2
    oracle.track_update(s, [108])            # x_hat 102.4, r 5.6: x 105.2, dx 0.96
    assert abs(s.x[0] - 105.2) < 1e-12 and abs(s.dx[0] - 0.96) < 1e-12
    assert s.frames == 3 and s.next_id == 1


def test_ramp_is_followed_without_lag():
    s = oracle.TrackState()
    for t in range(400):
        oracle.track_update(s, [200 + 3 * t])
    assert s.n == 1 and abs(s.x[0] - (200 + 3 * 399)) < 1e-9 and abs(s.dx[0] - 3.0) < 1e-9


def test_noise_variance_reduction_closed_form():
    """Steady-state position variance of an alpha-beta filter on white measurement noise:
    (2 beta + alpha (2 alpha - 3 beta)) / (alpha (4 - 2 alpha - beta)) of the noise variance."""
    a, b = 0.5, 0.1
    rng = np.random.default_rng(0)
    s = oracle.TrackState()
    xs = []
    for t in range(30000):
        oracle.track_update(s, [int(round(5000 + rng.normal(0.0, 6.0)))], gate=1e9)
        if t > 200:
            xs.append(s.x[0])
    meas_var = 36.0 + 1.0 / 12.0             # the rounding to whole columns adds 1/12
    ratio = np.var(xs) / meas_var
    want = (2 * b + a * (2 * a - 3 * b)) / (a * (4 - 2 * a - b))
    assert abs(ratio - want) < 0.05 * want, (ratio, want)


def test_gate_births_and_deaths():
    s = oracle.TrackState()
    for _ in range(4):
        oracle.track_update(s, [300])
    oracle.track_update(s, [330])            # 30 px > gate 24: a new track, the old one misses
    assert s.n == 2 and list(s.id[:2]) == [0, 1] and s.misses[0] == 1 and s.hits[1] == 1
    for k in range(5):                       # misses 2..6: dropped once misses > 5
        oracle.track_update(s, [330])
        assert (s.n == 2) == (k < 4)
    assert s.n == 1 and s.id[0] == 1 and s.hits[0] == 6
    assert [t[0] for t in s.tracks(confirm=3)] == [1]


def test_invalid_frames_and_capacity():
    s = oracle.TrackState()
    oracle.track_update(s, list(range(0, 2000, 100)))      # 20 detections: 16 tracks
    assert s.n == 16 and s.next_id == 16 and list(s.x[:16]) == [float(u) for u in range(0, 1600, 100)]
    oracle.track_update(s, [0, 100], valid=False)           # no road: every track misses
    assert all(s.misses[t] == 1 for t in range(16)) and s.n == 16


def test_closest_pair_first_and_ties():
    s = oracle.TrackState()
    oracle.track_update(s, [100, 120])                      # tracks 0 at 100, 1 at 120
    # 111 is 11 from track 0 and 9 from track 1; 104 is 4 from track 0: pairs by distance
    # (0,104) first, then (1,111)
    oracle.track_update(s, [111, 104])
    assert abs(s.x[0] - 102.0) < 1e-12 and abs(s.x[1] - 115.5) < 1e-12
    t = oracle.TrackState()
    oracle.track_update(t, [100, 110])
    oracle.track_update(t, [105])                           # 5 from both: the lower slot takes it
    assert t.misses[0] == 0 and t.misses[1] == 1
