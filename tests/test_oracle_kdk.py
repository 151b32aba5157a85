"""Pins of the kick-drift oracle and the Eq. 1 time step (Sec. 3.1).

  * a uniform acceleration is integrated exactly by kick-drift-kick leapfrog:
    after n steps x = x0 + v0 t + a t^2 / 2 and v = v0 + a t (to FP32 rounding);
  * the periodic wrap lands a particle leaving either face at the exact image;
  * zero kick and drift leave the state unchanged;
  * the per-cell rms velocity (mean not subtracted) and maximum acceleration
    equal numpy bincount / maximum.at over numpy floors of the positions;
  * Eq. 1 on hand-made statistics picks the Hubble limit, the coldest cell, or
    the global ratio when that is larger, as the paper describes.
"""
import math

import numpy as np
import pytest

import brute
import oracle
from paper_2110_11392_amd import synth


def test_uniform_acceleration_is_integrated_exactly():
    n, L = 64, 16.0
    rng = np.random.default_rng(11)
    x0 = (rng.random((n, 3)) * 4 + 6).astype(np.float32)
    v0 = (rng.standard_normal((n, 3))).astype(np.float32)
    g = np.array([0.5, -0.25, 0.125], np.float32)
    acc = np.tile(g, (n, 1)).astype(np.float32)
    dt, steps = 0.125, 16
    x, v = x0.copy(), v0.copy()
    # KDK: half kick, then (drift, full kick) repeated, the last kick halved
    _, v, _, _ = oracle.kick_drift(x, v, acc, L, 4, dt / 2, 0.0)
    for k in range(steps):
        x, v, _, _ = oracle.kick_drift(x, v, acc, L, 4, 0.0, dt)
        x, v, _, _ = oracle.kick_drift(x, v, acc, L, 4, dt if k < steps - 1 else dt / 2, 0.0)
    t = dt * steps
    xe = x0.astype(np.float64) + v0 * t + 0.5 * g.astype(np.float64) * t * t
    ve = v0.astype(np.float64) + g * t
    # one FP32 rounding per update: at most 2 * steps half-ulps of |x| < 16
    assert np.allclose(v, ve, rtol=0, atol=2 * steps * 2.0 ** -22)
    assert np.allclose(x, xe, rtol=0, atol=2 * steps * 2.0 ** -20)


@pytest.mark.parametrize("x,v,d,expect", [
    (0.9375, 0.25, 0.5, 0.0625),       # leaves the upper face
    (0.0625, -0.25, 0.5, 0.9375),      # leaves the lower face
    (0.5, 1.0, 3.0, 0.5),              # three whole boxes
    (0.75, 0.5, 0.5, 0.0),             # lands exactly on L -> 0
])
def test_drift_wraps_periodically(x, v, d, expect):
    pos = np.array([[x, 0.5, 0.5]], np.float32)
    vel = np.array([[v, 0.0, 0.0]], np.float32)
    acc = np.zeros((1, 3), np.float32)
    po, vo, _, _ = oracle.kick_drift(pos, vel, acc, 1.0, 4, 0.0, d)
    assert po[0, 0] == np.float32(expect)
    assert 0.0 <= po[0, 0] < 1.0
    assert np.array_equal(vo, vel)


def test_zero_step_is_identity():
    pos = synth.clustered(2000, 5, 8, 12)
    vel = synth.gaussian_weights(2000, 13)
    acc = synth.gaussian_weights(2000, 14)
    po, vo, _, _ = oracle.kick_drift(pos, vel, acc, 1.0, 8, 0.0, 0.0)
    assert np.array_equal(po, pos)
    assert np.array_equal(vo, vel)


def test_cell_statistics_match_numpy():
    n, K, L = 5000, 6, 2.0
    pos = synth.clustered(n, 7, K, 15, L)
    vel = synth.gaussian_weights(n, 16)
    acc = synth.gaussian_weights(n, 17) * np.float32(3.0)
    po, vo, cs, bs = oracle.kick_drift(pos, vel, acc, L, K, 0.01, 0.003)
    c = brute.cells(pos, L, K)
    cell = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    v2 = np.sum(vo.astype(np.float64) ** 2, axis=1)
    cnt = np.bincount(cell, minlength=K ** 3)
    vrms = np.sqrt(np.bincount(cell, weights=v2, minlength=K ** 3) / np.maximum(cnt, 1))
    amag = np.linalg.norm(acc.astype(np.float64), axis=1)
    amax = np.zeros(K ** 3)
    np.maximum.at(amax, cell, amag)
    assert np.allclose(cs[:, 0], vrms, rtol=1e-13, atol=0)
    assert np.allclose(cs[:, 1], amax, rtol=1e-15, atol=0)
    keep = (cnt > 0) & (amax > 0)
    assert bs[0] == pytest.approx(np.min(vrms[keep] / amax[keep]), rel=1e-13)
    assert bs[1] == pytest.approx(math.sqrt(v2.sum() / n), rel=1e-13)
    assert bs[2] == amag.max()
    assert bs[3] == n
    # the velocities are kicked, the positions drifted with the kicked velocities
    ve = (vel.astype(np.float64) + 0.01 * acc.astype(np.float64)).astype(np.float32)
    assert np.array_equal(vo, ve)
    xe = np.mod(pos.astype(np.float64) + 0.003 * vo.astype(np.float64), L).astype(np.float32)
    xe[xe >= np.float32(L)] = 0
    assert np.array_equal(po, xe)


def test_timestep_eq1_cases():
    # Hubble limit: eta_H a = 0.03 * 0.5 = 0.015 < accel step
    assert oracle.timestep([10.0, 1.0, 1.0, 100], 0.5, 2.0, 0.25, 0.03) == pytest.approx(0.015)
    # the coldest cell sets the step: 0.25 * 0.5 * 2 * 0.02 = 0.005
    assert oracle.timestep([0.02, 1.0, 100.0, 100], 0.5, 2.0, 0.25, 0.03) == pytest.approx(0.005)
    # an abnormally cold cell: the global ratio 1/10 is larger and is used,
    # 0.25 * 0.5 * 2 * 0.1 = 0.025 (below the Hubble limit 0.1 * 0.5)
    assert oracle.timestep([1e-6, 1.0, 10.0, 100], 0.5, 2.0, 0.25, 0.1) == pytest.approx(0.025)
    # no acceleration at all: only the Hubble limit remains
    assert oracle.timestep([math.inf, 1.0, 0.0, 100], 0.5, 2.0, 0.25, 0.03) == pytest.approx(0.015)


def test_kick_drift_rejects_bad_input():
    p = synth.uniform(10, 1)
    with pytest.raises(ValueError):
        oracle.kick_drift(p, p[:5], p, 1.0, 4, 0.1, 0.1)
    with pytest.raises(oracle.OracleError):
        oracle.kick_drift(p, p, p, 1.0, 4, float("nan"), 0.1)
