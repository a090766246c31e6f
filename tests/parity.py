"""Comparison helpers between the HIP path and the oracle (test infrastructure).

Tolerances (float parts), from the accuracy targets of the method:
  received power  <= 0.01 dB (P_inc, and P_coh when P_coh >= 1e-3 P_inc;
                  otherwise |dH| <= 1e-3 sqrt(P_inc / P_tx)),
  delay           <= 1e-9 relative,
  Doppler         <= 1e-6 Hz.
RMS delay spread <= 1e-9 of the mean delay; departure / arrival angles <= 1e-6
rad (the library reports them in float32).
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


def channel_ok(g: dict, o: dict, links: np.ndarray, p_tx: float, fi=None):
    """Check the channel tolerances on the given links at carrier fi (every
    carrier when fi is None): P_inc, P_coh (or H when the coherent sum is far
    below the incoherent one), mean delay and RMS delay spread (1e-9 of the
    mean delay), mean Doppler shift and RMS Doppler spread (1e-6 Hz).
    Returns the list of failures (link, quantity, carrier, gpu, oracle)."""
    bad = []
    carriers = range(np.asarray(o["P_inc"]).shape[0]) if fi is None else [fi]
    for f in carriers:
        for L in links:
            pi_g, pi_o = g["P_inc"][f][L], o["P_inc"][f][L]
            if pi_o == 0 and pi_g == 0:
                continue
            if not (pi_o > 0 and pi_g > 0) or db_err(pi_g, pi_o) > DB_TOL:
                bad.append((int(L), "P_inc", f, pi_g, pi_o))
                continue
            pc_g, pc_o = g["P_coh"][f][L], o["P_coh"][f][L]
            if pc_o >= 1e-3 * pi_o:
                if db_err(pc_g, pc_o) > DB_TOL:
                    bad.append((int(L), "P_coh", f, pc_g, pc_o))
            else:
                if abs(g["H"][f][L] - o["H"][f][L]) > 1e-3 * np.sqrt(pi_o / p_tx):
                    bad.append((int(L), "H", f, g["H"][f][L], o["H"][f][L]))
            tm = o["tau_mean"][f][L]
            for name in ("tau_mean", "tau_rms"):
                if abs(g[name][f][L] - o[name][f][L]) > TAU_REL * tm:
                    bad.append((int(L), name, f, g[name][f][L], o[name][f][L]))
            for name in ("fd_mean", "fd_rms"):
                if abs(g[name][f][L] - o[name][f][L]) > FD_ABS:
                    bad.append((int(L), name, f, g[name][f][L], o[name][f][L]))
    return bad


def compare_angles(g_ang: np.ndarray, o_aod: np.ndarray, o_aoa: np.ndarray, tol: float = 1e-6) -> float:
    """Largest difference between the library's float32 angles [n, 4] (AoD az,
    el, AoA az, el) and the oracle's double ones, azimuths wrapped; the
    library rounds the double angle to float32 (<= 2.4e-7 rad)."""
    o = np.concatenate([np.asarray(o_aod), np.asarray(o_aoa)], axis=1)
    d = np.asarray(g_ang, np.float64) - o
    d[:, [0, 2]] = (d[:, [0, 2]] + np.pi) % (2 * np.pi) - np.pi
    return float(np.max(np.abs(d))) if len(d) else 0.0


def gpu_channels_np(ch: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in ch.items()}


def compare_captures(rows: np.ndarray, tx: int, ray_ids: np.ndarray, trace, strict: bool = True) -> tuple:
    """Per-ray capture sets of the GPU's capture log (rows of tx, launch
    direction, bounce, kind, id) against an oracle ``TraceResult`` of the
    same directions of transmitter tx.  strict: every row of tx must belong
    to one of ray_ids (else rows of other marked directions are skipped).
    Returns (robust rays compared, rays whose receiver or edge capture set
    differs)."""
    rows = np.asarray(rows).reshape(-1, 5)
    rows = rows[rows[:, 0] == tx]
    pos = {int(r): k for k, r in enumerate(ray_ids)}
    g_rx = [set() for _ in ray_ids]
    g_ed = [set() for _ in ray_ids]
    for _, d, b, kind, i in rows:
        k = pos.get(int(d))
        if k is None:
            assert not strict, f"capture of an unmarked direction {d}"
            continue
        (g_ed if kind == 1 else g_rx)[k].add((int(b), int(i)))
    o_rx = [set() for _ in ray_ids]
    o_ed = [set() for _ in ray_ids]
    for k, b, r in trace.captures:
        o_rx[k].add((int(b), int(r)))
    for k, e, b in trace.edge_hits:
        o_ed[k].add((int(b), int(e)))
    bad = [k for k in range(len(ray_ids)) if trace.robust[k] and (g_rx[k] != o_rx[k] or g_ed[k] != o_ed[k])]
    return int(trace.robust.sum()), bad
