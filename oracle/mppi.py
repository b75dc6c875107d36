"""FP64 CPU oracle of the sampled-rollout controller -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product path never does.

The paper's obstacle-avoidance showcase (section "Model Predictive Path
Integral" of the Methods, and the MPPI paragraph of the Results) runs several
independent sampling controllers that are a hybrid of iCEM and MPPI: each one
samples temporally correlated command sequences around its previous mean
(warm start), rolls every sample through the full simulator, keeps the best
1 % of the samples (elites), and forms the new mean as an exponentially
weighted average of the elites; the controller with the best sample supplies
the command. The paper leaves the cost, the noise colour, the temperature and
the other hyper-parameters to a codebase that is not part of it. Readings taken
here (one each, stated where they are used):

  m1  noise: standard normals from the counter-based Philox4x64-10 generator
      (Salmon et al., SC'11) with counter (block, sample, controller, iteration)
      and key (seed, 0), turned into normals by the Box-Muller transform; one
      generator block (four 64-bit words, eight 32-bit halves) gives the four
      command components of two consecutive horizon steps;
  m2  temporal correlation: a first-order autoregressive filter with unit
      stationary variance, eps_0 = xi_0, eps_t = beta eps_{t-1} + sqrt(1 -
      beta^2) xi_t (iCEM uses power-law coloured noise; this is the one-pole
      version of the same idea);
  m3  sample 0 of every controller is the (shifted) mean itself, noise-free;
  m4  command = clip(mean + sigma * eps, u_lo, u_hi) per component;
  m5  cost = sum over the horizon of r_u |u_t - u_ref|^2 (diagonal) on the
      applied commands plus q_p |p - goal|^2 + q_v |v|^2 + w_obs * sum_o
      max(0, 1 - |p - c_o|^2 / r_o^2)^2 on the states after each command; a
      non-finite cost counts as +infinity;
  m6  elites: the n_e samples of lowest cost, ties broken by the lower sample
      index; weights exp(-(J - J_min) / lambda) over the elites only;
  m7  warm start: the mean read at horizon index min(t + shift, H - 1);
  m8  selection among controllers: the lowest elite cost, ties to the lower
      controller index; the command applied is that controller's new mean at
      horizon step 0.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from .dynamics import MODEL_FP, Batch

# ---- Philox4x64-10 (published definition) -------------------------------------

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def _mulhilo64(a: int, b: np.ndarray):
    """(hi, lo) 64-bit halves of the 128-bit product a * b, b a uint64 array."""
    a0, a1 = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (p00 & _M32)
    return hi, lo


def philox4x64(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x64 with 10 rounds: ctr ``[..., 4]`` uint64, key (k0, k1) ->
    ``[..., 4]`` uint64. Each round multiplies words 0 and 2 by the two round
    constants, mixes the high halves with words 1 and 3 and the key, and the key
    is bumped by the two Weyl constants between rounds."""
    x = [np.ascontiguousarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFFFFFFFFFF, int(key[1]) & 0xFFFFFFFFFFFFFFFF
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = (k0 + PHILOX_W0) & 0xFFFFFFFFFFFFFFFF
                k1 = (k1 + PHILOX_W1) & 0xFFFFFFFFFFFFFFFF
            hi0, lo0 = _mulhilo64(PHILOX_M0, x[0])
            hi1, lo1 = _mulhilo64(PHILOX_M1, x[2])
            x = [hi1 ^ x[1] ^ np.uint64(k0), lo1, hi0 ^ x[3] ^ np.uint64(k1), lo0]
    return np.stack(x, -1)


def uniform_from_u32(u: np.ndarray) -> np.ndarray:
    """Open-interval uniform (0, 1) from the top 23 bits: ((u >> 9) + 1/2) 2^-23
    (exact in binary32 and binary64)."""
    return ((u.astype(np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def normals_from_block(words: np.ndarray) -> np.ndarray:
    """Eight standard normals from one generator block ``[..., 4]`` uint64 (m1):
    the 32-bit halves (low, high) of each word form a Box-Muller pair,
    z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)."""
    lo = (words & _M32).astype(np.uint64)
    hi = (words >> _S32).astype(np.uint64)
    u1, u2 = uniform_from_u32(lo), uniform_from_u32(hi)
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.stack([r * np.cos(2 * math.pi * u2), r * np.sin(2 * math.pi * u2)], -1)   # [..., 4, 2]
    return z.reshape(*words.shape[:-1], 8)


def white_noise(ctrl: np.ndarray, sample: np.ndarray, H: int, seed: int, iteration: int) -> np.ndarray:
    """xi ``[n, H, 4]`` for the (controller, sample) pairs given (m1)."""
    n = len(ctrl)
    nb = (H + 1) // 2
    ctr = np.zeros((n, nb, 4), np.uint64)
    ctr[..., 0] = np.arange(nb, dtype=np.uint64)[None, :]
    ctr[..., 1] = np.asarray(sample, np.uint64)[:, None]
    ctr[..., 2] = np.asarray(ctrl, np.uint64)[:, None]
    ctr[..., 3] = np.uint64(iteration)
    z = normals_from_block(philox4x64(ctr, (seed, 0)))          # [n, nb, 8]
    return z.reshape(n, 2 * nb, 4)[:, :H]


def correlated_noise(ctrl, sample, H, seed, iteration, beta) -> np.ndarray:
    """eps ``[n, H, 4]``: the autoregressive filter of m2, zero for sample 0 (m3)."""
    xi = white_noise(np.asarray(ctrl), np.asarray(sample), H, seed, iteration)
    eps = np.empty_like(xi)
    g = math.sqrt(1.0 - beta * beta)
    eps[:, 0] = xi[:, 0]
    for t in range(1, H):
        eps[:, t] = beta * eps[:, t - 1] + g * xi[:, t]
    eps[np.asarray(sample) == 0] = 0.0
    return eps


def shifted_mean(mean: np.ndarray, shift: int) -> np.ndarray:
    """Warm start (m7): mean ``[C, H, 4]`` read at min(t + shift, H - 1)."""
    H = mean.shape[1]
    return mean[:, np.minimum(np.arange(H) + shift, H - 1)]


def sample_commands(mean_s: np.ndarray, ctrl, eps: np.ndarray, P: Dict) -> np.ndarray:
    """u ``[n, H, 4]`` = clip(mean + sigma eps, u_lo, u_hi) (m4)."""
    u = mean_s[np.asarray(ctrl)] + np.asarray(P["sigma"])[None, None, :] * eps
    return np.clip(u, np.asarray(P["u_lo"]), np.asarray(P["u_hi"]))


def rollout_costs(w, x_now: np.ndarray, u: np.ndarray, P: Dict) -> np.ndarray:
    """Cost of m5 for each command sequence u ``[n, H, 4]`` started at x_now ``[S]``
    on the single world of workload ``w`` (its model, interface, integrator,
    dt, controller period), with ``substeps`` simulator steps per horizon step;
    the onboard controller's blocks count physics steps from the first one."""
    n, H, _ = u.shape
    batch = Batch([n], w.model_per_world[:1], {k: v[:1] for k, v in w.params.items()}, w.control,
                  w.integrator, w.dt, w.renorm_q, getattr(w, "ctrl_every", 1))
    x = torch.as_tensor(np.asarray(x_now, np.float64))[:, None].repeat(1, n)
    ut = torch.as_tensor(u, dtype=torch.float64)
    goal = torch.as_tensor(np.asarray(P["goal"], np.float64))[:, None]
    vrow = 7 if int(w.model_per_world[0]) == MODEL_FP else 6
    obs = np.asarray(P.get("obstacles", np.zeros((0, 4))), np.float64).reshape(-1, 4)
    r_u = torch.as_tensor(np.asarray(P["r_u"], np.float64))[:, None]
    u_ref = torch.as_tensor(np.asarray(P["u_ref"], np.float64))[:, None]
    J = torch.zeros(n, dtype=torch.float64)
    sub = int(P.get("substeps", 1))
    held = None
    with torch.no_grad():
        for t in range(H):
            ct = ut[:, t].T.contiguous()
            J = J + (r_u * (ct - u_ref) ** 2).sum(0)
            for k in range(sub):
                x, held = batch.step_at(x, ct, t * sub + k, held)
            p, v = x[0:3], x[vrow:vrow + 3]
            J = J + P["q_p"] * ((p - goal) ** 2).sum(0) + P["q_v"] * (v ** 2).sum(0)
            for o in obs:
                d2 = ((p - torch.as_tensor(o[:3])[:, None]) ** 2).sum(0)
                J = J + P["w_obs"] * torch.clamp(1.0 - d2 / (o[3] * o[3]), min=0.0) ** 2
    J = J.numpy()
    J[~np.isfinite(J)] = np.inf
    return J


def select_elites(J: np.ndarray, n_elite: int) -> np.ndarray:
    """Indices ``[C, n_e]`` of the n_e lowest costs per controller, ordered by
    (cost, sample index) (m6)."""
    C, N = J.shape
    out = np.empty((C, n_elite), np.int64)
    for c in range(C):
        order = np.lexsort((np.arange(N), J[c]))
        out[c] = order[:n_elite]
    return out


def elite_mean(u_elite: np.ndarray, J_elite: np.ndarray, lam: float) -> np.ndarray:
    """Exponentially weighted mean of the elites (m6): u_elite ``[n_e, H, 4]``,
    J_elite ``[n_e]`` ascending."""
    wgt = np.exp(-(J_elite - J_elite[0]) / lam)
    return (wgt[:, None, None] * u_elite).sum(0) / wgt.sum()


def mppi_step(w, P: Dict, x_now: np.ndarray, mean: np.ndarray, shift: int, iteration: int,
              costs: Optional[np.ndarray] = None, elites: Optional[np.ndarray] = None) -> Dict:
    """One control step of all controllers. ``costs`` / ``elites`` replace the
    oracle's own (used to check a device's selection and weighted mean given
    the device's FP32 costs, where the decision between near-equal costs is
    the device's)."""
    C, H, _ = mean.shape
    N, n_e = int(P["n_samples"]), int(P["n_elite"])
    ms = shifted_mean(np.asarray(mean, np.float64), shift)
    if costs is None:
        cc, kk = np.repeat(np.arange(C), N), np.tile(np.arange(N), C)
        eps = correlated_noise(cc, kk, H, P["seed"], iteration, P["beta"])
        u = sample_commands(ms, cc, eps, P)
        costs = rollout_costs(w, x_now, u, P).reshape(C, N)
    J = np.asarray(costs, np.float64)
    if elites is None:
        elites = select_elites(J, n_e)
    new_mean = np.empty((C, H, 4))
    for c in range(C):
        k = elites[c]
        eps = correlated_noise(np.full(n_e, c), k, H, P["seed"], iteration, P["beta"])
        ue = sample_commands(ms, np.full(n_e, c), eps, P)
        new_mean[c] = elite_mean(ue, J[c, k], P["lambda"])
    jmin = J[np.arange(C), elites[:, 0]]
    best = int(np.lexsort((np.arange(C), jmin))[0])
    return {"costs": J, "elites": elites, "cost_min": jmin, "mean": new_mean, "best": best,
            "u_apply": new_mean[best, 0].copy()}
