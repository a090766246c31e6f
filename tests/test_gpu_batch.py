"""Batched stepping (emrt_batch) vs stepping each scene alone.

Several uneven cities of the 64-city batched workload (moving vehicles, 1-3
transmitters, K = 4) are stepped through a schedule of discovery and cached
frames twice: once with one context per city stepped alone, and once as a
batch (multi-scene persistent bounce launches, HIP-graph replay).  Every
replay is checked against the separate steps, with eager host work and
synchronisations in between.  The per-city results are deterministic, so
channels and path lists must be identical.  The batched results are also
checked against the oracle itself: sampled paths of every city validate in it
with the same gains, delays and Doppler shifts, and the channel sums of its
links equal the oracle's sums over the same keys.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402
from tests import parity as P  # noqa: E402

pytestmark = pytest.mark.gpu

CITIES = (44, 9, 29, 34, 20, 4)  # the smallest of the 64 (75k-117k rays each)
SCHEDULE = (True, False, False, True, False, True)


def _tracer(w, **kw):
    from paper_2303_10521_amd import Tracer

    sc = w.scene
    args = dict(freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=w.rays_per_tx,
                diffraction=int(w.diffraction), path_capacity=1 << 20)
    args.update(kw)
    return Tracer(sc, sc.n_tx, sc.n_rx, **args)


def _snapshot(tr):
    ch = tr.channels()
    out = {k: ch[k].cpu().numpy().copy() for k in ("H", "P_coh", "P_inc", "tau_mean", "fd_mean", "fd_rms", "n_paths")}
    p = tr.flat_paths(cap=64)
    out["keys"] = p["key"].copy()
    return out


def _equal(a, b):
    for k in a:
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k


def _run_schedule(use_graph, n_streams, grid, ks=None, chunk=64):
    from paper_2303_10521_amd import Batch

    ws = [city.batch_city(i) for i in CITIES]
    if ks is not None:
        for w, k in zip(ws, ks):
            w.max_reflections = k
    solo = [_tracer(w) for w in ws]
    members = [_tracer(w) for w in ws]
    batch = Batch(members, use_graph=use_graph, n_streams=n_streams, grid=grid, chunk=chunk)
    for f, disc in enumerate(SCHEDULE):
        for w, a, b in zip(ws, solo, members):
            fr = w.scene.frame(f * w.frame_dt)
            a.set_frame(fr, f)
            b.set_frame(fr, f)
            a.step(disc)
        batch.step(disc)
        assert batch.sync() == 0
        for a, b in zip(solo, members):
            assert a.sync() == 0
            _equal(_snapshot(a), _snapshot(b))
    batch.close()
    for t in solo + members:
        t.close()


def test_batch_graph_replays_match_separate_steps():
    _run_schedule(True, 4, 2048)


def test_batch_eager_single_stream_matches_separate_steps():
    _run_schedule(False, 1, 512)


def test_batch_mixed_bounce_depths():
    _run_schedule(True, 2, 1024, ks=(4, 2, 4, 3, 0, 4))


@pytest.mark.parametrize("chunk", [32, 128, 256, 1024])
def test_batch_chunk_sizes_match_separate_steps(chunk):
    """Every chunk size of the multi-scene bounce (half-wave chunks of 32
    rays, two and four passes of 64) gives the separate steps' results."""
    _run_schedule(True, 4, 2048, chunk=chunk)


def test_batch_rules_and_autotune(tmp_path):
    from paper_2303_10521_amd import Batch
    from paper_2303_10521_amd.tracer import EmrtError

    ws = [city.batch_city(i) for i in CITIES[:3]]
    members = [_tracer(w) for w in ws]
    batch = Batch(members)
    with pytest.raises(EmrtError):
        batch.step(True)  # no frames yet
    for w, t in zip(ws, members):
        t.set_frame(w.scene.frame(0.0))
    with pytest.raises(EmrtError):
        members[0].step(True)  # members step through the batch only
    with pytest.raises(EmrtError):
        Batch([members[0]])  # already batched
    with pytest.raises(EmrtError):
        batch.set_options(True, 4, 2048, chunk=48)  # not a supported chunk size
    cache = str(tmp_path / "tune.json")
    o = batch.autotune(repeats=1, cache=cache)
    assert not o["from_cache"] and o["key"].startswith("gfx950|")
    assert o["grid"] in (1024, 2048, 4096, 8192) and o["streams"] in (1, 2, 4, 8) and o["chunk"] in (64, 128, 256, 512)
    again = batch.autotune(repeats=1, cache=cache)  # the cached shape, no timing
    assert again["from_cache"] and {k: again[k] for k in ("grid", "streams", "chunk")} == {
        k: o[k] for k in ("grid", "streams", "chunk")}
    batch.step(True)
    assert batch.sync() == 0
    batch.close()
    for t in members:
        t.close()


def test_members_step_alone_and_rebatch_after_close():
    """A closed batch gives its members their own streams back: each steps
    alone again with the results of a never-batched context, and the same
    members form a new batch (the first batch's stream is gone by then)."""
    import gc

    from paper_2303_10521_amd import Batch

    ws = [city.batch_city(i) for i in CITIES[:3]]
    members = [_tracer(w) for w in ws]
    solo = [_tracer(w) for w in ws]
    for w, t, s in zip(ws, members, solo):
        fr = w.scene.frame(0.0)
        t.set_frame(fr)
        s.set_frame(fr)
    b1 = Batch(members, n_streams=2)
    b1.step(True)
    assert b1.sync() == 0
    for s in solo:
        s.step(True)
    b1.close()
    del b1
    gc.collect()  # the first batch's stream is released
    for w, t, s in zip(ws, members, solo):
        fr = w.scene.frame(w.frame_dt)
        t.set_frame(fr, 1)
        s.set_frame(fr, 1)
        t.step(True)
        s.step(True)
        assert t.sync() == 0 and s.sync() == 0
        _equal(_snapshot(s), _snapshot(t))
    b2 = Batch(members, n_streams=4, chunk=32)
    for w, t in zip(ws, members):
        t.set_frame(w.scene.frame(2 * w.frame_dt), 2)
    b2.step(True)
    assert b2.sync() == 0
    b2.close()
    for t in members + solo:
        t.close()


def _oracle_check_member(w, tr, fr, n_pick=300, n_links=120, seed=0):
    """Sampled paths and per-link sums of one batch member against the oracle."""
    sc = w.scene
    os_ = O.OracleScene(sc)
    g = os_.geometry(fr.obj_xform)
    p = tr.flat_paths(cap=256)
    ch = P.gpu_channels_np(tr.channels())
    assert not p["truncated"]
    keys = p["key"]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(keys), min(n_pick, len(keys)), replace=False)
    valid, amb, tri, pts = O.validate(os_, g, keys[pick], fr.tx_pos, fr.rx_pos)
    assert np.all(valid | amb)
    ok = valid & ~amb
    assert ok.sum() >= 0.95 * len(pick)
    a, tau, fd, aod, aoa = O.evaluate(os_, g, keys[pick][ok], pts[ok], fr, w.freqs_hz)
    assert np.all(np.abs(p["a"][pick][ok] - a) <= 1e-8 * np.abs(a))
    assert np.all(np.abs(p["tau"][pick][ok] - tau) <= P.TAU_REL * tau)
    assert np.all(np.abs(p["fd"][pick][ok] - fd) <= P.FD_ABS)
    assert P.compare_angles(p["angles"][pick][ok], aod, aoa) <= 1e-6
    spec = keys[pick][ok][:, 2] == 1
    assert np.array_equal(p["tri_ids"][pick][ok][spec], tri[ok][spec])
    # channel sums over every path of sampled links
    link = keys[:, 0].astype(np.int64) * sc.n_rx + keys[:, 1]
    have = np.unique(link)
    links = rng.choice(have, min(n_links, len(have)), replace=False)
    sel = np.isin(link, links)
    valid, amb, tri, pts = O.validate(os_, g, keys[sel], fr.tx_pos, fr.rx_pos)
    assert np.all(valid | amb)
    a, tau, fd, _, _ = O.evaluate(os_, g, keys[sel], pts, fr, w.freqs_hz)
    ref = O.reduce_links(keys[sel], a, tau, fd, sc.n_tx, sc.n_rx)
    amb_links = set(link[sel][amb].tolist())
    check = np.array([L for L in links if L not in amb_links])
    assert len(check) >= 0.8 * len(links)
    assert not P.channel_ok(ch, ref, check, 100.0)
    return len(pick), len(check)


def test_batch_cities_against_oracle():
    """The batched form itself against the oracle: after graph-replayed
    discovery, cached and discovery frames, every city's sampled paths and
    link sums agree with the oracle at that frame."""
    from paper_2303_10521_amd import Batch

    ws = [city.batch_city(i) for i in CITIES]
    members = [_tracer(w) for w in ws]
    batch = Batch(members, use_graph=True, n_streams=4, grid=2048)
    n_paths = n_links = 0
    for f, disc in enumerate((True, False, True)):
        frs = [w.scene.frame(f * w.frame_dt) for w in ws]
        for t, fr in zip(members, frs):
            t.set_frame(fr, f)
        batch.step(disc)
        assert batch.sync() == 0
        for i, (w, t, fr) in enumerate(zip(ws, members, frs)):
            a, b = _oracle_check_member(w, t, fr, seed=10 * f + i)
            n_paths += a
            n_links += b
    assert n_paths >= 3 * 300 * len(CITIES) * 0.5 and n_links >= 3 * 90 * len(CITIES)
    batch.close()
    for t in members:
        t.close()
