"""Sampled-rollout controller on the GPU vs the FP64 oracle, through the C ABI:
the correlated noise, per-sample costs, the elite set (decided on the device's
own FP32 costs, where the oracle must pick exactly the same samples), the
weighted mean, the controller choice, and the argument checks."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import dev
from oracle import mppi as OM
from paper_2606_01478_amd import binding as B

pytestmark = pytest.mark.gpu


def _make(model=W.MODEL_FP, C=3, N=2000, H=25, **over):
    w, P, mean0 = W.mppi_task(n_controllers=C, n_samples=N, horizon=H, model=model)
    P.update(over)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    return w, P, mean0, sim, B.Mppi(sim, P)


def _jittered_mean(mean0, seed=0):
    rng = np.random.default_rng(seed)
    m = mean0.astype(np.float64).copy()
    m[..., 0:2] += rng.normal(0, 0.1, size=m[..., 0:2].shape)
    m[..., 3] *= rng.uniform(0.95, 1.1, size=m[..., 3].shape)
    return m.astype(np.float32)


def _run(w, P, mp, mean, shift, it):
    C, N, H, ne = P["n_controllers"], P["n_samples"], P["horizon"], P["n_elite"]
    x_now = dev(w.x0[:, 0])
    m = dev(mean)
    out = dict(u=torch.empty(4, device="cuda"), best=torch.empty(1, dtype=torch.int32, device="cuda"),
               cost=torch.empty((C, N), device="cuda"), el=torch.empty((C, ne), dtype=torch.int32, device="cuda"),
               cmin=torch.empty(C, device="cuda"))
    mp.step(x_now, m, shift, it, u_apply=out["u"], best=out["best"], cost=out["cost"], elite_idx=out["el"],
            cost_min=out["cmin"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()} | {"mean": m.cpu().numpy()}


def _check_step(w, P, mean, shift, it, got, sample=None):
    C, N = P["n_controllers"], P["n_samples"]
    ms = OM.shifted_mean(mean.astype(np.float64), shift)
    # costs (all samples, or a sample of them)
    if sample is None:
        cc, kk = np.repeat(np.arange(C), N), np.tile(np.arange(N), C)
    else:
        cc, kk = sample
    eps = OM.correlated_noise(cc, kk, P["horizon"], P["seed"], it, P["beta"])
    u = OM.sample_commands(ms, cc, eps, P)
    Jr = OM.rollout_costs(w, w.x0[:, 0], u, P)
    Jg = got["cost"][cc, kk].astype(np.float64)
    rel = np.abs(Jg - Jr) / np.abs(Jr)
    assert rel.max() <= 1e-4, rel.max()
    # elites: the oracle's selection on the device's own costs picks the same samples
    Jd = got["cost"].astype(np.float64)
    el = OM.select_elites(Jd, P["n_elite"])
    assert np.array_equal(got["el"], el)
    assert np.array_equal(got["cmin"].astype(np.float64), Jd[np.arange(C), el[:, 0]])
    # weighted mean from the same elites and costs, FP64 commands
    ref = OM.mppi_step(w, P, w.x0[:, 0], mean, shift, it, costs=Jd, elites=el)
    scale = np.asarray(P["sigma"]) + np.abs(ms).max(axis=(0, 1))
    err = np.abs(got["mean"] - ref["mean"]) / scale
    assert err.max() <= 1e-4, err.max()
    assert int(got["best"][0]) == ref["best"]
    assert np.array_equal(got["u"], got["mean"][ref["best"], 0])


def test_noise_matches_oracle(gpu_lib):
    w, P, mean0, sim, mp = _make(C=2, N=300, H=25)
    eps = torch.empty((2, 300, 25, 4), device="cuda")
    mp.noise(3, eps)
    torch.cuda.synchronize()
    cc, kk = np.repeat(np.arange(2), 300), np.tile(np.arange(300), 2)
    ref = OM.correlated_noise(cc, kk, 25, P["seed"], 3, P["beta"]).reshape(2, 300, 25, 4)
    g = eps.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - ref) <= 1e-5 * (1 + np.abs(ref)))
    assert np.all(g[:, 0] == 0)


@pytest.mark.parametrize("model", [W.MODEL_FP, W.MODEL_ID])
def test_step_matches_oracle(gpu_lib, model):
    w, P, mean0, sim, mp = _make(model=model)
    mean = _jittered_mean(mean0, 1)
    got = _run(w, P, mp, mean, 1, 7)
    _check_step(w, P, mean, 1, 7, got)


def test_substeps_and_odd_horizon(gpu_lib):
    w, P, mean0, sim, mp = _make(C=2, N=700, H=13, substeps=3, n_elite=9)
    mean = _jittered_mean(mean0, 2)
    got = _run(w, P, mp, mean, 0, 0)
    _check_step(w, P, mean, 0, 0, got)


def test_repeatable_and_improving(gpu_lib):
    """The same (seed, iteration) gives the same bits; iterating with the warm
    start lowers the best cost of the no-obstacle task."""
    w, P, mean0, sim, mp = _make(C=2, N=4000, H=20, n_obstacles=0, n_elite=40)
    a = _run(w, P, mp, mean0, 0, 11)
    b = _run(w, P, mp, mean0, 0, 11)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    mean = mean0
    first = None
    for it in range(6):
        r = _run(w, P, mp, mean, 1 if it else 0, it)
        mean = r["mean"]
        first = r["cmin"].min() if first is None else first
    assert r["cmin"].min() < first


def test_zero_noise_ties(gpu_lib):
    """sigma = 0: every sample is the mean, all costs are equal, the elites are the
    lowest sample indices and the plan is the shifted mean."""
    w, P, mean0, sim, mp = _make(C=2, N=500, H=9, sigma=[0.0] * 4, n_elite=17)
    mean = _jittered_mean(mean0, 3)
    got = _run(w, P, mp, mean, 2, 5)
    assert np.all(got["cost"] == got["cost"][:, :1])
    assert np.array_equal(got["el"], np.tile(np.arange(17), (2, 1)))
    ms = np.clip(OM.shifted_mean(mean.astype(np.float64), 2), P["u_lo"], P["u_hi"])
    assert np.allclose(got["mean"], ms, rtol=1e-6, atol=1e-7)


def test_full_size_500k_samples(gpu_lib):
    """5 controllers x 100 000 samples x 25 steps: 256 sampled costs against the
    oracle, the whole elite selection and the weighted means."""
    w, P, mean0, sim, mp = _make(C=5, N=100_000, H=25)
    mean = _jittered_mean(mean0, 4)
    got = _run(w, P, mp, mean, 1, 2)
    rng = np.random.default_rng(5)
    cc, kk = rng.integers(0, 5, 256), rng.integers(0, 100_000, 256)
    kk[:5], cc[:5] = 0, np.arange(5)
    _check_step(w, P, mean, 1, 2, got, sample=(cc, kk))


def test_rejects_invalid_arguments(gpu_lib):
    w, P, mean0 = W.mppi_task(n_controllers=2, n_samples=100, horizon=5)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    for bad in (dict(n_elite=0), dict(n_elite=101), dict(beta=1.0), dict(lambda_=0.0), dict(horizon=0),
                dict(substeps=0), dict(u_lo=[1.0, 0, 0, 0], u_hi=[0.0, 0, 0, 0])):
        Q = dict(P)
        if "lambda_" in bad:
            Q["lambda"] = bad.pop("lambda_")
        Q.update(bad)
        with pytest.raises(B.CfError):
            B.Mppi(sim, Q)
    obs = np.array([[0, 0, 1, 0.0]], np.float32)
    with pytest.raises(B.CfError):
        B.Mppi(sim, dict(P, obstacles=obs))
    w2 = W.fp_pid_closed_loop(seed=1, n_worlds=2, steps=1)
    with pytest.raises(B.CfError):
        B.Mppi(B.Sim.from_workload(w2, flags=B.F_NO_AUTOTUNE_CACHE), P)
    mp = B.Mppi(sim, P)
    host = np.zeros((2, P["horizon"], 4), np.float32)     # not device memory
    st = gpu_lib.cf_mppi_step(mp._m, dev(w.x0[:, 0]).data_ptr(), host.ctypes.data, 0, 0, None, None, None, None,
                              None)
    assert st == B.CF_EINVAL
    st = gpu_lib.cf_mppi_step(mp._m, dev(w.x0[:, 0]).data_ptr(), dev(mean0).data_ptr(), -1, 0, None, None, None,
                              None, None)
    assert st == B.CF_EINVAL
    assert sim.last_error() == 0


@pytest.mark.parametrize("N,n_e,sigma0", [(8000, 3000, False), (5000, 40, True), (3000, 1500, False)])
def test_selection_paths(gpu_lib, N, n_e, sigma0):
    """Both selection paths (sampled threshold for n_e <= 2048, radix select above)
    pick exactly the oracle's elites from the device's costs, also with ties."""
    over = dict(n_elite=n_e)
    if sigma0:
        over["sigma"] = [0.0] * 4
    w, P, mean0, sim, mp = _make(C=2, N=N, H=6, **over)
    got = _run(w, P, mp, _jittered_mean(mean0, 7), 1, 3)
    Jd = got["cost"].astype(np.float64)
    assert np.array_equal(got["el"], OM.select_elites(Jd, n_e))
    assert np.array_equal(got["cmin"].astype(np.float64), Jd[np.arange(2), got["el"][:, 0]])


def test_diverging_samples_count_as_infinite(gpu_lib):
    """Samples whose rollout overflows get an infinite cost and never become
    elites; the plan stays finite."""
    w, P, mean0, sim, mp = _make(model=W.MODEL_ID, C=2, N=3000, H=8, n_elite=20,
                                 sigma=[0.15, 0.15, 0.3, 3e37], u_hi=[0.6, 0.6, 3.2, 3.4e38])
    got = _run(w, P, mp, mean0, 0, 4)
    J = got["cost"]
    assert np.isinf(J).any() and np.isfinite(J).any()
    assert not np.isnan(J).any()
    assert np.all(np.isfinite(J[np.arange(2)[:, None], got["el"]]))
    assert np.array_equal(got["el"], OM.select_elites(J.astype(np.float64), 20))
    assert np.all(np.isfinite(got["mean"]))
