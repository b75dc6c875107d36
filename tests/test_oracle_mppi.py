"""Pins of the sampled-rollout controller oracle against facts that do not come
from the oracle itself: numpy's own Philox4x64-10, the moments of the normal and
autoregressive noise, brute-force sorting, limits of the weighted mean and a
closed-form cost."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mppi as OM


def _np_philox_blocks(counter, key, n):
    """numpy's Philox bit generator advances the counter before each block, so
    its first block is the one for counter + 1."""
    bg = np.random.Philox(counter=np.array(counter, np.uint64), key=np.array(key, np.uint64))
    return bg.random_raw(4 * n).reshape(n, 4)


def _inc(ctr, by):
    """256-bit little-endian counter increment."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr)) + by
    v &= (1 << 256) - 1
    return [(v >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)]


@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 7, 11, 13], [0x0123456789ABCDEF, 0xFEDCBA9876543210]),
    ([2 ** 64 - 3, 2 ** 64 - 1, 17, 0], [2 ** 64 - 1, 2 ** 64 - 1]),   # carries across words
    ([123456789, 0, 3, 2 ** 63], [42, 0]),
])
def test_philox_matches_numpy(counter, key):
    n = 9
    ref = _np_philox_blocks(counter, key, n)
    ctr = np.array([_inc(counter, i + 1) for i in range(n)], np.uint64)
    got = OM.philox4x64(ctr, key)
    assert np.array_equal(got, ref.astype(np.uint64))


def test_uniforms_are_exact_midpoints():
    u = np.array([0, 1 << 9, 0xFFFFFFFF, 0x80000000], np.uint64)
    x = OM.uniform_from_u32(u)
    assert np.array_equal(x, np.array([0.5, 1.5, 2 ** 23 - 0.5, 2 ** 22 + 0.5]) * 2.0 ** -23)
    assert np.all((x > 0) & (x < 1))
    # every value is exact in binary32
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)


def test_normals_moments_and_independence():
    n = 200_000
    z = OM.white_noise(np.zeros(n, np.int64), np.arange(n), 4, seed=99, iteration=1)   # [n, 4, 4]
    f = z.reshape(-1)
    assert abs(f.mean()) < 4 * 1 / math.sqrt(f.size)
    assert abs(f.var() - 1) < 6 * math.sqrt(2 / f.size)
    # fourth moment of a standard normal is 3
    assert abs((f ** 4).mean() - 3) < 0.03
    # components and steps are uncorrelated
    c = np.corrcoef(z.reshape(n, 16).T)
    assert np.max(np.abs(c - np.eye(16))) < 0.02
    # tail: P(|z| > 3) = 0.0027
    assert abs((np.abs(f) > 3).mean() - 0.0026998) < 0.0006


@pytest.mark.parametrize("beta", [0.0, 0.8, 0.95])
def test_autoregressive_noise_covariance(beta):
    """Unit stationary variance at every step and Corr(eps_t, eps_{t+s}) = beta^s."""
    n, H = 100_000, 9
    eps = OM.correlated_noise(np.zeros(n, np.int64), np.arange(1, n + 1), H, seed=5, iteration=0, beta=beta)
    e = eps[:, :, 1]
    var = e.var(0)
    assert np.max(np.abs(var - 1)) < 0.03
    for s in (1, 2, 4):
        r = np.mean([np.corrcoef(e[:, t], e[:, t + s])[0, 1] for t in range(H - s)])
        assert abs(r - beta ** s) < 0.02, (s, r)


def test_sample_zero_is_the_mean():
    eps = OM.correlated_noise(np.array([0, 0, 1]), np.array([0, 3, 0]), 5, seed=1, iteration=2, beta=0.5)
    assert np.all(eps[0] == 0) and np.all(eps[2] == 0) and np.any(eps[1] != 0)


def test_elite_selection_brute_force():
    rng = np.random.default_rng(0)
    J = np.round(rng.uniform(0, 5, size=(3, 400)), 1)   # many ties
    J[1, 7] = np.inf
    el = OM.select_elites(J, 37)
    for c in range(3):
        ref = [k for _, k in sorted((J[c, k], k) for k in range(400))][:37]
        assert list(el[c]) == ref


def test_weighted_mean_limits():
    rng = np.random.default_rng(1)
    u = rng.normal(size=(20, 6, 4))
    J = np.sort(rng.uniform(0, 10, 20))
    assert np.allclose(OM.elite_mean(u, J, 1e12), u.mean(0), rtol=0, atol=1e-9)
    assert np.allclose(OM.elite_mean(u, J, 1e-3), u[0], rtol=0, atol=1e-12)
    # shift invariance of the cost
    assert np.allclose(OM.elite_mean(u, J, 2.0), OM.elite_mean(u, J + 100.0, 2.0), rtol=0, atol=1e-12)


def test_cost_closed_form_at_hover():
    """A hovering drone (noise-free commands equal to hover) stays put, so every
    term of the cost is constant: J = H (q_p |p0 - g|^2 + w (1 - d^2/r^2)^2)."""
    w, P, mean0 = W.mppi_task(n_controllers=1, n_samples=1, horizon=6)
    p0 = w.x0[0:3, 0].astype(np.float64)
    P = dict(P, obstacles=np.array([[p0[0] + 0.1, p0[1], p0[2], 0.3]], np.float32), r_u=[1.0, 1.0, 1.0, 1.0])
    u = np.repeat(mean0[0:1].astype(np.float64), 1, 0)    # [1, H, 4]
    J = OM.rollout_costs(w, w.x0[:, 0], u, P)[0]
    g = np.asarray(P["goal"])
    r = float(np.float32(0.3))
    pen = (1 - 0.1 ** 2 / r ** 2) ** 2
    expect = 6 * (P["q_p"] * ((p0 - g) ** 2).sum() + P["w_obs"] * pen)
    assert abs(J - expect) < 1e-7 * expect


def test_zero_noise_is_a_fixed_point():
    """sigma = 0: all samples equal the shifted mean, all costs tie, the elites are
    the lowest indices and the new mean is the shifted (clipped) mean."""
    w, P, mean0 = W.mppi_task(n_controllers=2, n_samples=40, horizon=7)
    P = dict(P, sigma=[0.0] * 4, n_elite=5)
    rng = np.random.default_rng(2)
    mean = mean0.astype(np.float64) + rng.normal(0, 0.01, size=mean0.shape)
    r = OM.mppi_step(w, P, w.x0[:, 0], mean, 2, 0)
    assert np.all(r["costs"] == r["costs"][:, :1])
    assert np.array_equal(r["elites"], np.tile(np.arange(5), (2, 1)))
    ms = np.clip(OM.shifted_mean(mean, 2), P["u_lo"], P["u_hi"])
    assert np.allclose(r["mean"], ms, rtol=0, atol=1e-15)


def test_iterations_lower_the_best_cost():
    w, P, mean0 = W.mppi_task(n_controllers=2, n_samples=400, horizon=15, n_obstacles=0)
    P = dict(P, n_elite=8)
    mean = mean0.astype(np.float64)
    first = None
    for it in range(5):
        r = OM.mppi_step(w, P, w.x0[:, 0], mean, 0, it)
        mean = r["mean"]
        first = r["cost_min"].min() if first is None else first
    assert r["cost_min"].min() < first
