"""Standard particle filter weights and residual resampling (the SIR comparison filter).

Paper: Section "Standard particle filter" -- w_i proportional to exp(-1/2 d^T R^{-1} d)
(eq. standardParticleFilterWeight), resampled with residual resampling (Liu & Chen):
each particle is first copied floor(N_e w_i) times, the remaining N_e - sum floor(N_e w_i)
slots are drawn multinomially from the residual weights N_e w_i - floor(N_e w_i).

Reading (exact, order-fixed so that integer results are reproducible):
  e_i = exp(l_i - max l) with l the natural log-weights, S = sum_i e_i left to right,
  n_i = floor(N_e e_i / S), r_i = N_e e_i / S - n_i, residual draws k = 0.. by inverse CDF
  over the left-to-right cumulative sum of r_i against u_k * sum(r) with
  u_k = uniform k of the stream (tag RESAMPLE).  Parents are returned sorted ascending.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox


def sir_log_weights(d: np.ndarray, sigma: float) -> np.ndarray:
    """l_i = -1/2 sum_o |d_io|^2 / sigma^2 for innovations d [Ne, n_obs, 2]."""
    return -0.5 * np.sum(d * d, axis=(1, 2)) / (sigma * sigma)


def residual_resample(logw: np.ndarray, uniforms: np.ndarray):
    """Returns (parents int32 [Ne] ascending, counts int64 [Ne])."""
    ne = len(logw)
    m = max(float(v) for v in logw)
    e = [math.exp(float(v) - m) for v in logw]
    s = 0.0
    for v in e:
        s += v
    counts = np.zeros(ne, dtype=np.int64)
    resid = []
    for i in range(ne):
        x = ne * e[i] / s
        n = math.floor(x)
        counts[i] = n
        resid.append(x - n)
    n_res = ne - int(counts.sum())
    cum = []
    acc = 0.0
    for v in resid:
        acc += v
        cum.append(acc)
    total = acc
    for k in range(n_res):
        target = uniforms[k] * total
        pick = ne - 1
        for i in range(ne):
            if target < cum[i]:
                pick = i
                break
        counts[pick] += 1
    parents = np.repeat(np.arange(ne, dtype=np.int32), counts)
    return parents, counts


def resample_uniforms(ne: int, seed: int, analysis_index: int, ensemble_id: int) -> np.ndarray:
    return philox.uniforms(ne, seed, analysis_index, philox.TAG_RESAMPLE, ensemble_id, 0)
