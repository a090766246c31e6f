"""Coherence statistics on the GPU (emrt_read_coherence) vs the oracle.

The toy city with its street receivers moving at 8-15 m/s, stepped with
discovery every third frame and cache revalidation in between, on both the
GPU and the oracle.  Compared per link: the spatial-consistency triggers
(exactly), Eq (2)'s coherence time (to 1e-12) and Eq (1)'s lagged
autocovariance of |H| (to 1e-6 where the variance is not a rounding
residue).  Links whose path sets ever differ between the two are left out.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import coherence as Co  # noqa: E402
from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402

pytestmark = pytest.mark.gpu

R = 0.5
LAGS = [1, 2, 3, 4]


def _moving_toy():
    w = city.workload("toy")
    sc = w.scene
    ped = {k: np.array(v, copy=True) for k, v in sc.rx_ped.items()}
    n = len(ped["vel"])
    ped["vel"] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * (8.0 + 7.0 * (np.arange(n) % 3) / 2.0)
    return w, dataclasses.replace(sc, rx_ped=ped)


def _keysets(keys, n_rx):
    out = {}
    for k in np.asarray(keys).reshape(-1, 9):
        out.setdefault(int(k[0]) * n_rx + int(k[1]), set()).add(tuple(int(x) for x in k))
    return out


def test_coherence_matches_oracle_over_frames():
    from paper_2303_10521_amd import Tracer

    w, sc = _moving_toy()
    n_rx, nl = sc.n_rx, sc.n_tx * sc.n_rx
    tr = Tracer(sc, sc.n_tx, n_rx, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections,
                rays_per_tx=w.rays_per_tx, path_capacity=1 << 16)
    os_ = O.OracleScene(sc)
    ok_links = np.ones(nl, bool)
    g_hist, prev_los, prev_sets, cache = [], None, None, None
    for f in range(9):
        fr = sc.frame(0.2 * f)
        disc = f % 3 == 0
        tr.set_frame(fr, f)
        tr.step(disc)
        assert tr.sync() == 0
        got = tr.coherence(R)
        ref = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, list(w.freqs_hz), discover=disc, cache=cache)
        cache = O.cache_of(ref)
        gk = _keysets(tr.flat_paths(cap=256)["key"], n_rx)
        rk = _keysets(ref.keys, n_rx)
        for l in range(nl):
            if gk.get(l, set()) != rk.get(l, set()):
                ok_links[l] = False
        # oracle statistics
        los = ref.channels["los"]
        sets = Co.first_order_sets(ref.keys, nl, n_rx)
        trig = Co.triggers(prev_los, los, prev_sets, sets)
        prev_los, prev_sets = los, sets
        g_hist.append(np.abs(ref.channels["H"]))  # [nf, nl]
        corr = Co.autocovariance(np.array(g_hist), LAGS)  # [lags, nf, nl]
        tx_i = np.arange(nl) // n_rx
        rx_i = np.arange(nl) % n_rx
        v_rel = fr.rx_vel[rx_i] - fr.tx_vel[tx_i]
        d = fr.rx_pos[rx_i] - fr.tx_pos[tx_i]
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        tc = np.array([Co.coherence_time(R, fq, v_rel, d) for fq in w.freqs_hz])
        # compare
        gt = got["trigger"].cpu().numpy().astype(np.uint32)
        assert np.array_equal(gt[ok_links], trig[ok_links]), f
        gtc = got["tc"].cpu().numpy()
        fin = np.isfinite(tc)
        assert np.array_equal(np.isfinite(gtc), fin)
        assert np.allclose(gtc[fin], tc[fin], rtol=1e-12, atol=0)
        gc = got["corr"].cpu().numpy()  # [nf, nl, lags]
        ref_c = np.transpose(corr, (1, 2, 0))
        g = np.array(g_hist)
        var = (g * g).mean(0) - g.mean(0) ** 2
        well = (var > 1e-6 * g.mean(0) ** 2) & ok_links[None, :]
        for k in range(len(LAGS)):
            a, b = gc[..., k][well], ref_c[..., k][well]
            assert np.array_equal(np.isnan(a), np.isnan(b)), (f, k)
            m = ~np.isnan(a)
            assert np.allclose(a[m], b[m], atol=1e-6, rtol=0), (f, k)
        finite = tc[fin]
        want_min = finite.min() if finite.size else np.inf
        assert got["min_tc"] == want_min or abs(got["min_tc"] - want_min) <= 1e-12 * want_min
        assert got["n_triggered"] == int((gt != 0).sum())
    assert ok_links.mean() >= 0.9
    # a reset starts a new segment: no triggers, undefined correlations
    tr.coherence_reset()
    tr.set_frame(sc.frame(2.0), 9)
    tr.step(False)
    got = tr.coherence(R)
    assert int(got["trigger"].abs().sum()) == 0
    assert torch.isnan(got["corr"]).all()
    tr.close()
