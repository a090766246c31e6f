"""Comparison helpers between the HIP path and the oracle (test infrastructure).

Tolerances (float parts), from the accuracy targets of the method:
  received power  <= 0.01 dB (P_inc, and P_coh when P_coh >= 1e-3 P_inc;
                  otherwise |dH| <= 1e-3 sqrt(P_inc / P_tx)),
  delay           <= 1e-9 relative,
  Doppler         <= 1e-6 Hz.
Interaction sequences (triangle ids per bounce) are compared bit-exactly on
rays the oracle marks robust; path sets are compared exactly except for keys
whose discovery or validation the oracle marks ambiguous.
"""
from __future__ import annotations

import numpy as np

DB_TOL = 0.01
TAU_REL = 1e-9
FD_ABS = 1e-6


def keyset(keys) -> set:
    return {tuple(int(x) for x in k) for k in np.asarray(keys).reshape(-1, 9)}


def compare_hitlogs(gpu_hits: np.ndarray, oracle_hits: np.ndarray, robust: np.ndarray):
    """Returns (n_robust, n_mismatch_on_robust, n_mismatch_total)."""
    eq = np.all(gpu_hits == oracle_hits, axis=1)
    return int(robust.sum()), int((~eq & robust).sum()), int((~eq).sum())


def db_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(10 * np.log10(a / b))


def compare_path_values(gk, gp, ok, op, nf):
    """Per-path complex gain, delay and Doppler of common keys.
    gp / op: dicts with a [n, nf], tau [n], fd [n, nf]; gk/ok keys [n, 9]."""
    gi = {tuple(int(x) for x in k): i for i, k in enumerate(gk)}
    worst = {"a_rel": 0.0, "tau_rel": 0.0, "fd_abs": 0.0, "n": 0}
    for j, k in enumerate(ok):
        i = gi.get(tuple(int(x) for x in k))
        if i is None:
            continue
        worst["n"] += 1
        ga, oa = np.asarray(gp["a"][i]).reshape(nf), np.asarray(op["a"][j]).reshape(nf)
        worst["a_rel"] = max(worst["a_rel"], float(np.max(np.abs(ga - oa) / np.maximum(np.abs(oa), 1e-300))))
        worst["tau_rel"] = max(worst["tau_rel"], abs(gp["tau"][i] - op["tau"][j]) / op["tau"][j])
        worst["fd_abs"] = max(worst["fd_abs"], float(np.max(np.abs(np.asarray(gp["fd"][i]).reshape(nf) -
                                                                 np.asarray(op["fd"][j]).reshape(nf)))))
    return worst


def channel_ok(g: dict, o: dict, links: np.ndarray, p_tx: float, fi: int = 0):
    """Check channel tolerances on the given links; returns list of failures."""
    bad = []
    for L in links:
        pi_g, pi_o = g["P_inc"][fi][L], o["P_inc"][fi][L]
        if pi_o == 0 and pi_g == 0:
            continue
        if not (pi_o > 0 and pi_g > 0) or db_err(pi_g, pi_o) > DB_TOL:
            bad.append((int(L), "P_inc", pi_g, pi_o))
            continue
        pc_g, pc_o = g["P_coh"][fi][L], o["P_coh"][fi][L]
        if pc_o >= 1e-3 * pi_o:
            if db_err(pc_g, pc_o) > DB_TOL:
                bad.append((int(L), "P_coh", pc_g, pc_o))
        else:
            if abs(g["H"][fi][L] - o["H"][fi][L]) > 1e-3 * np.sqrt(pi_o / p_tx):
                bad.append((int(L), "H", g["H"][fi][L], o["H"][fi][L]))
        if abs(g["tau_mean"][fi][L] - o["tau_mean"][fi][L]) > TAU_REL * o["tau_mean"][fi][L]:
            bad.append((int(L), "tau_mean", g["tau_mean"][fi][L], o["tau_mean"][fi][L]))
        if abs(g["fd_mean"][fi][L] - o["fd_mean"][fi][L]) > FD_ABS:
            bad.append((int(L), "fd_mean", g["fd_mean"][fi][L], o["fd_mean"][fi][L]))
        if abs(g["fd_rms"][fi][L] - o["fd_rms"][fi][L]) > FD_ABS:
            bad.append((int(L), "fd_rms", g["fd_rms"][fi][L], o["fd_rms"][fi][L]))
    return bad


def gpu_channels_np(ch: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in ch.items()}
