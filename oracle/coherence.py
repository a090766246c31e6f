"""Oracle of the coherence statistics (Section III-B): TEST INFRASTRUCTURE ONLY.

Only ``tests/`` import this module.  Plain numpy over per-frame oracle
results; it shares nothing with the GPU library.

Readings (the paper gives the formulas but not their estimators):
* Eq (1), the channel correlation of g(t) = |h(t)|, has a garbled
  denominator; it is read as the normalised autocovariance
      R(k) = (E[g_t g_{t-k}] - E[g]^2) / (E[g^2] - E[g]^2),
  estimated over the frames seen so far at lags of k frames:
      E[g_t g_{t-k}] = mean over t = k..n-1 of g_t g_{t-k},
      E[g] = mean of g_0..g_{n-1},  E[g^2] = mean of g_t^2,
  undefined (NaN) while n <= k or the variance is zero.
* Eq (2), the coherence time T_c(theta) = sqrt(1/R^4 - 1) / (2 pi f_D theta^2),
  with R the correlation threshold (default 0.5), f_D = f_c |v| / c the
  largest Doppler shift of the link's relative velocity v = v_rx - v_tx, and
  theta the acute angle between the line of motion and the transmitter ->
  receiver direction; +inf when f_D theta^2 = 0.
* Spatial-consistency triggers (the trajectory segmentation of Section
  III-A): per link, bit 0 when the line-of-sight flag differs from the
  previous frame's, bit 1 when the set of first-order paths (one
  reflection or one diffraction) differs.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

C0 = 299792458.0


def coherence_time(R: float, f_c: float, v_rel: np.ndarray, k_dir: np.ndarray) -> np.ndarray:
    """Eq (2) per link: v_rel [n, 3] relative velocities, k_dir [n, 3] unit
    transmitter -> receiver directions."""
    v = np.linalg.norm(v_rel, axis=1)
    f_d = f_c * v / C0
    with np.errstate(invalid="ignore", divide="ignore"):
        cosang = np.abs(np.sum(v_rel * k_dir, axis=1)) / np.where(v > 0, v, 1.0)
    theta = np.arccos(np.clip(cosang, 0.0, 1.0))
    den = 2.0 * math.pi * f_d * theta * theta
    num = math.sqrt(1.0 / R ** 4 - 1.0)
    with np.errstate(divide="ignore"):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), np.inf)


def autocovariance(g: np.ndarray, lags: Sequence[int]) -> np.ndarray:
    """Eq (1) as read above for a series g [n_frames, ...]; returns
    [len(lags), ...] (NaN where undefined)."""
    g = np.asarray(g, np.float64)
    n = g.shape[0]
    m = g.mean(axis=0)
    var = (g * g).mean(axis=0) - m * m
    out = []
    for k in lags:
        if n <= k:
            out.append(np.full(g.shape[1:], np.nan))
            continue
        c = (g[k:] * g[:-k]).mean(axis=0) - m * m
        with np.errstate(invalid="ignore", divide="ignore"):
            out.append(np.where(var != 0, c / np.where(var != 0, var, 1.0), np.nan))
    return np.array(out)


def first_order_sets(keys: np.ndarray, n_links: int, n_rx: int) -> list:
    """Per link, the set of first-order path keys (order-1 specular or diffraction)."""
    sets = [frozenset() for _ in range(n_links)]
    acc: Dict[int, set] = {}
    for k in np.asarray(keys).reshape(-1, 9):
        if int(k[3]) == 1 and int(k[2]) in (1, 2):
            acc.setdefault(int(k[0]) * n_rx + int(k[1]), set()).add(tuple(int(x) for x in k))
    for l, s in acc.items():
        sets[l] = frozenset(s)
    return sets


def triggers(prev_los: Optional[np.ndarray], los: np.ndarray, prev_sets: Optional[list], sets: list) -> np.ndarray:
    """Spatial-consistency trigger bits per link (0 on the first frame)."""
    t = np.zeros(len(los), np.uint32)
    if prev_los is None:
        return t
    t |= (np.asarray(prev_los, bool) != np.asarray(los, bool)).astype(np.uint32)
    t |= np.array([2 if a != b else 0 for a, b in zip(prev_sets, sets)], np.uint32)
    return t
