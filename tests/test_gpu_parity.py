"""HIP path vs the FP64 oracle, through the C ABI.

Levels of comparison:
  * per ray: triangle id per bounce, bit-exact on rays the oracle marks robust
    (every decision farther than its margin from a boundary);
  * per link: path-key sets equal except keys the oracle marks ambiguous;
  * per path and per link: gain, delay and Doppler within the tolerances of
    tests/parity.py.
The toy city is compared in full; the district and the 2x2 km city run at
their full sizes in the benchmark's launch configuration and are compared on
sampled rays, sampled keys and sampled links that the oracle computes one by
one.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402
from tests import parity as P  # noqa: E402
from tests.oracle_util import static_frame  # noqa: E402

pytestmark = pytest.mark.gpu


def _tracer(sc, w, **kw):
    from paper_2303_10521_amd import Tracer

    args = dict(freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=w.rays_per_tx,
                diffraction=int(w.diffraction), path_capacity=1 << 22)
    args.update(kw)
    return Tracer(sc, sc.n_tx, sc.n_rx, **args)


# ---------------------------------------------------------------- toy city
@pytest.fixture(scope="module")
def toy():
    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    tr = _tracer(sc, w, path_capacity=1 << 16)
    tr.set_frame(fr)
    tr.step(True)
    assert tr.sync() == 0
    out = dict(w=w, sc=sc, fr=fr, tr=tr,
               hits=tr.debug_rays(0, np.arange(w.rays_per_tx)),
               paths=tr.flat_paths(), ch=P.gpu_channels_np(tr.channels()))
    os_ = O.OracleScene(sc)
    out["os"] = os_
    out["ref"] = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, w.freqs_hz)
    yield out
    tr.close()


def test_toy_interaction_sequences_bit_exact(toy):
    t0 = toy["ref"].traces[0]
    n_rob, mm_rob, mm_all = P.compare_hitlogs(toy["hits"], t0.hit_tri, t0.robust)
    assert n_rob >= 0.98 * len(t0.robust)
    assert mm_rob == 0
    assert mm_all <= len(t0.robust) - n_rob


def test_toy_path_sets(toy):
    ref = toy["ref"]
    g = P.keyset(toy["paths"]["key"])
    unamb = P.keyset(ref.keys[~ref.ambiguous & ref.robust])
    assert unamb <= g
    extra = np.array(sorted(g - P.keyset(ref.keys)), np.int32).reshape(-1, 9)
    if len(extra):
        valid, amb, _, _ = O.validate(toy["os"], toy["os"].geometry(toy["fr"].obj_xform), extra,
                                      toy["fr"].tx_pos, toy["fr"].rx_pos)
        assert np.all(valid | amb)
    assert len(extra) <= max(1, len(g) // 50)


def test_toy_path_values_and_triangles(toy):
    ref, p = toy["ref"], toy["paths"]
    gi = {tuple(int(x) for x in k): i for i, k in enumerate(p["key"])}
    n = 0
    for j, k in enumerate(ref.keys):
        i = gi.get(tuple(int(x) for x in k))
        if i is None:
            continue
        n += 1
        assert abs(p["a"][i, 0] - ref.a[j, 0]) <= 1e-8 * abs(ref.a[j, 0])
        assert abs(p["tau"][i] - ref.tau[j]) <= P.TAU_REL * ref.tau[j]
        assert abs(p["fd"][i, 0] - ref.fd[j, 0]) <= P.FD_ABS
        if not ref.ambiguous[j]:
            assert np.array_equal(p["tri_ids"][i], ref.tri_ids[j])
        assert P.compare_angles(p["angles"][i][None], ref.aod[j][None], ref.aoa[j][None]) <= 1e-6
    assert n >= 0.95 * len(ref.keys)


def test_toy_channels(toy):
    ref = toy["ref"]
    g = toy["ch"]
    links = np.arange(toy["sc"].n_rx)
    assert not P.channel_ok(g, ref.channels, links, 100.0)
    assert np.array_equal(g["n_paths"], ref.channels["n_paths"])
    assert np.array_equal(g["flags"] & 1, ref.channels["los"].astype(np.int32))


def test_toy_dipole_forward_values():
    """Dipole transmitters (antenna mode 1) at a tilted orientation, with
    diffraction, at two carriers: per-path complex gains, delays and
    Dopplers, and every link's channels, against the oracle's dipole
    evaluation (the isotropic runs do not reach the pattern terms)."""
    from paper_2303_10521_amd import Tracer

    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    fr.tx_orient = np.array([[0.6, 0.4]])
    freqs = [3.5e9, 28e9]
    tr = Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=freqs, max_reflections=w.max_reflections, rays_per_tx=w.rays_per_tx,
                diffraction=1, antenna_mode=1, path_capacity=1 << 16)
    try:
        tr.set_frame(fr)
        tr.step(True)
        assert tr.sync() == 0
        os_ = O.OracleScene(sc)
        ref = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, freqs, diffraction=True, ant_mode=1)
        iso = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, freqs, diffraction=True, ant_mode=0)
        assert np.abs(ref.a - iso.a).max() > 0.1 * np.abs(iso.a).max()  # the pattern matters here
        assert set(np.unique(ref.keys[:, 2]).tolist()) == {0, 1, 2}
        p = tr.flat_paths(cap=256)
        worst = P.compare_path_values(p["key"], p, ref.keys, dict(a=ref.a, tau=ref.tau, fd=ref.fd), len(freqs))
        assert worst["n"] >= 0.95 * len(ref.keys)
        assert worst["a_rel"] <= 1e-8 and worst["tau_rel"] <= P.TAU_REL and worst["fd_abs"] <= P.FD_ABS, worst
        g = P.keyset(p["key"])
        mask = np.ones(sc.n_tx * sc.n_rx, bool)
        for k in g ^ P.keyset(ref.keys):
            mask[k[0] * sc.n_rx + k[1]] = False
        assert mask.mean() >= 0.9
        assert not P.channel_ok(P.gpu_channels_np(tr.channels()), ref.channels, np.nonzero(mask)[0], 100.0)
    finally:
        tr.close()


def test_toy_deterministic_and_cached_frame(toy):
    tr, fr = toy["tr"], toy["fr"]
    tr.set_frame(fr)
    tr.step(True)
    again = P.gpu_channels_np(tr.channels())
    for k in again:
        assert np.array_equal(again[k], toy["ch"][k]), k
    tr.step(False)  # static scene: the cache reproduces the same channels
    cached = P.gpu_channels_np(tr.channels())
    for k in cached:
        assert np.array_equal(cached[k], toy["ch"][k]), k


# ------------------------------------------------ district at full size
@pytest.fixture(scope="module")
def district():
    w = city.workload("district")
    sc = w.scene
    tr = _tracer(sc, w, path_capacity=1 << 23)
    frames = [sc.frame(i * w.frame_dt) for i in range(4)]
    out = dict(w=w, sc=sc, tr=tr, frames=frames, os=O.OracleScene(sc))
    tr.set_frame(frames[0], 0)
    tr.step(True)
    assert tr.sync() == 0
    out["hits"] = {t: tr.debug_rays(t, np.arange(t, w.rays_per_tx, 509)) for t in range(sc.n_tx)}
    out["paths"] = tr.flat_paths(cap=256)
    out["ch"] = P.gpu_channels_np(tr.channels())
    out["cache0"] = tr.cache_export()
    yield out
    tr.close()


def test_district_sampled_rays_bit_exact(district):
    w, sc, fr = district["w"], district["sc"], district["frames"][0]
    os_ = district["os"]
    g = os_.geometry(fr.obj_xform)
    tot = 0
    for t in range(sc.n_tx):
        ids = np.arange(t, w.rays_per_tx, 509, dtype=np.int32)
        res = O.trace(os_, g, fr.tx_pos[t], w.rays_per_tx, ids, w.max_reflections, fr.rx_pos, 1.0, True, True)
        n_rob, mm_rob, _ = P.compare_hitlogs(district["hits"][t], res.hit_tri, res.robust)
        assert mm_rob == 0
        assert n_rob >= 0.95 * len(ids)
        tot += len(ids)
    assert tot > 7000


def test_district_paths_exact_in_oracle(district):
    """Sampled GPU paths (specular and diffraction) validate in the oracle with
    the same triangles, gains, delays and Doppler shifts."""
    fr = district["frames"][0]
    os_ = district["os"]
    p = district["paths"]
    assert not p["truncated"]
    keys = p["key"]
    rng = np.random.default_rng(0)
    types = keys[:, 2]
    assert (types == 2).sum() > 100 and (types == 1).sum() > 100
    pick = np.concatenate([rng.choice(np.nonzero(types == t)[0], min(400, (types == t).sum()), replace=False)
                           for t in (0, 1, 2)])
    g = os_.geometry(fr.obj_xform)
    valid, amb, tri, pts = O.validate(os_, g, keys[pick], fr.tx_pos, fr.rx_pos)
    assert np.all(valid | amb)
    assert valid.mean() > 0.99
    ok = valid & ~amb
    a, tau, fd, aod, aoa = O.evaluate(os_, g, keys[pick][ok], pts[ok], fr, district["w"].freqs_hz)
    ga = p["a"][pick][ok]
    assert np.all(np.abs(ga - a) <= 1e-8 * np.abs(a))
    assert P.compare_angles(p["angles"][pick][ok], aod, aoa) <= 1e-6
    assert np.all(np.abs(p["tau"][pick][ok] - tau) <= P.TAU_REL * tau)
    assert np.all(np.abs(p["fd"][pick][ok] - fd) <= P.FD_ABS)
    spec = keys[pick][ok][:, 2] == 1
    assert np.array_equal(p["tri_ids"][pick][ok][spec], tri[ok][spec])


def test_district_channel_sums(district):
    """Per-link sums over the GPU's path set equal the oracle's sums over the
    same keys (sampled links, every path of the link)."""
    fr = district["frames"][0]
    os_ = district["os"]
    sc = district["sc"]
    p = district["paths"]
    link = p["key"][:, 0] * sc.n_rx + p["key"][:, 1]
    rng = np.random.default_rng(1)
    links = rng.choice(np.unique(link), 150, replace=False)
    sel = np.isin(link, links)
    keys = p["key"][sel]
    g = os_.geometry(fr.obj_xform)
    valid, amb, tri, pts = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos)
    assert np.all(valid | amb)
    a, tau, fd, _, _ = O.evaluate(os_, g, keys, pts, fr, district["w"].freqs_hz)
    ref = O.reduce_links(keys, a, tau, fd, sc.n_tx, sc.n_rx)
    # links with an ambiguous path are excluded (their oracle sum is undefined here)
    amb_links = set(link[sel][amb].tolist())
    check = np.array([L for L in links if L not in amb_links])
    assert len(check) > 100
    assert not P.channel_ok(district["ch"], ref, check, 100.0)


def test_district_discovery_covers_oracle_subset(district):
    """Keys the oracle discovers robustly from a launch subset (every 53rd ray
    of every transmitter) and validates unambiguously are all in the GPU set,
    which traces every ray."""
    w, sc, fr = district["w"], district["sc"], district["frames"][0]
    os_ = district["os"]
    ids = np.arange(0, w.rays_per_tx, 53, dtype=np.int32)
    ref = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, w.freqs_hz, ray_ids=ids, diffraction=False)
    spec = (ref.keys[:, 2] == 1) & ref.robust & ~ref.ambiguous
    want = P.keyset(ref.keys[spec])
    assert len(want) > 40
    assert want <= P.keyset(district["paths"]["key"])


def test_district_cached_frames_revalidate(district):
    """Cached frames keep only keys that are valid at the new geometry
    (deletion of invalid paths), never add keys, and agree with the oracle's
    validation of the same cache."""
    tr, os_, w = district["tr"], district["os"], district["w"]
    prev = P.keyset(district["cache0"])
    for f in (1, 2, 3):
        fr = district["frames"][f]
        tr.set_frame(fr, f)
        tr.step(False)
        assert tr.sync() == 0
        cache = tr.cache_export()
        cur = P.keyset(cache)
        assert cur <= prev
        dropped = np.array(sorted(prev - cur), np.int32).reshape(-1, 9)
        g = os_.geometry(fr.obj_xform)
        if len(dropped):
            valid, amb, _, _ = O.validate(os_, g, dropped, fr.tx_pos, fr.rx_pos)
            assert np.all(~valid | amb)
        rng = np.random.default_rng(f)
        keep = cache[rng.choice(len(cache), min(600, len(cache)), replace=False)]
        valid, amb, _, _ = O.validate(os_, g, keep, fr.tx_pos, fr.rx_pos)
        assert np.all(valid | amb)
        prev = cur
    # restore frame 0 state for other tests
    tr.set_frame(district["frames"][0], 0)
    tr.step(True)


def test_district_resume_from_exported_cache(district):
    """Checkpoint / resume: a fresh context that imports the exported cache
    produces the same cached-frame channels as the original context."""
    w, sc = district["w"], district["sc"]
    tr = district["tr"]
    fr1 = district["frames"][1]
    tr.set_frame(district["frames"][0], 0)
    tr.step(True)
    keys = tr.cache_export()
    tr.set_frame(fr1, 1)
    tr.step(False)
    a = P.gpu_channels_np(tr.channels())
    tr2 = _tracer(sc, w, path_capacity=1 << 23)
    tr2.cache_import(keys)
    tr2.set_frame(fr1, 1)
    tr2.step(False)
    b = P.gpu_channels_np(tr2.channels())
    tr2.close()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_district_static_reuse_equals_full_tests(district):
    """Cached frames reuse the last step's tests against the static scene for
    keys whose end points did not move (static receivers, and every key when
    a frame is stepped twice).  A context that imports the same cache has no
    last step and tests everything in full: channels and the next cache are
    identical, frame after frame."""
    w, sc = district["w"], district["sc"]
    tr = district["tr"]
    tr.set_frame(district["frames"][0], 0)
    tr.step(True)
    tr2 = _tracer(sc, w, path_capacity=1 << 23)
    for f in (1, 2, 2, 3):  # frame 2 twice: nothing moves between those steps
        keys = tr.cache_export()
        fr = district["frames"][f]
        tr.set_frame(fr, f)
        tr.step(False)
        assert tr.sync() == 0
        tr2.cache_import(keys)
        tr2.set_frame(fr, f)
        tr2.step(False)
        assert tr2.sync() == 0
        a, b = P.gpu_channels_np(tr.channels()), P.gpu_channels_np(tr2.channels())
        for k in a:
            assert np.array_equal(a[k], b[k]), (f, k)
        assert P.keyset(tr.cache_export()) == P.keyset(tr2.cache_export()), f
    tr2.close()
    tr.set_frame(district["frames"][0], 0)
    tr.step(True)


# ------------------------------------------- 2x2 km city at full size
# The benchmark workload in the benchmark's launch configuration: 16 Tx x 1M
# rays, K = 5, first-order diffraction, 10k moving receivers, 3.5 and 28 GHz.
CITY_STRIDE = 7919  # every 7919th launch direction of every transmitter: 16 x 127 rays


@pytest.fixture(scope="module")
def city_run():
    w = city.workload("city")
    sc = w.scene
    # rays regrouped between bounces (ray_regroup = 1): the full-size frame checks
    # that path against the oracle, the other tests run the default append order
    tr = _tracer(sc, w, path_capacity=1 << 23, ray_regroup=1)
    fr = sc.frame(0.0)
    tr.set_frame(fr, 0)
    ids = {t: np.arange(t * 37, w.rays_per_tx, CITY_STRIDE, dtype=np.int32) for t in range(sc.n_tx)}
    cov_ids = np.arange(5, w.rays_per_tx, 256, dtype=np.int32)  # the discovery-coverage subset
    for t in range(sc.n_tx):  # the capture decisions of both subsets are logged
        tr.debug_select_rays(t, ids[t])
        tr.debug_select_rays(t, cov_ids)
    tr.step(True)
    assert tr.sync() == 0
    os_ = O.OracleScene(sc)
    out = dict(w=w, sc=sc, tr=tr, fr=fr, os=os_, g=os_.geometry(fr.obj_xform), stats=tr.stats())
    out["ids"] = ids
    out["cov_ids"] = cov_ids
    out["captures"] = tr.debug_ray_captures()
    out["hits"] = {t: tr.debug_rays(t, out["ids"][t]) for t in range(sc.n_tx)}
    out["paths"] = tr.flat_paths(cap=128)
    out["ch"] = P.gpu_channels_np(tr.channels())
    # the oracle's traces of the same launch directions (receiver and edge capture, robust-ray mask)
    out["traces"] = {t: O.trace(os_, out["g"], fr.tx_pos[t], w.rays_per_tx, out["ids"][t], w.max_reflections,
                                fr.rx_pos, 1.0, True, True) for t in range(sc.n_tx)}
    out["cov_traces"] = {t: O.trace(os_, out["g"], fr.tx_pos[t], w.rays_per_tx, cov_ids, w.max_reflections,
                                    fr.rx_pos, 1.0, True, True) for t in range(sc.n_tx)}
    yield out
    tr.close()


def test_city_sizes(city_run):
    st = city_run["stats"]
    assert st["n_edges"] == 36800 and st["rays_per_bounce"][0] == 16_000_000
    assert len(city_run["paths"]["key"]) == int(city_run["ch"]["n_paths"].sum()) or city_run["paths"]["truncated"]


def test_city_hit_logs_all_transmitters(city_run):
    """Per-ray interaction sequences, bit-exact on robust rays, for about 2,000
    launch directions spread over all 16 transmitters."""
    tot = rob = 0
    for t, res in city_run["traces"].items():
        n_rob, mm_rob, _ = P.compare_hitlogs(city_run["hits"][t], res.hit_tri, res.robust)
        assert mm_rob == 0, (t, mm_rob)
        tot += len(res.robust)
        rob += n_rob
    assert tot >= 2000 and rob >= 0.9 * tot


def test_city_capture_sets_per_ray(city_run):
    """Receiver captures (reception spheres on the segments after a
    reflection) and edge captures (first segment) ray by ray: on every robust
    ray of both sampled subsets (about 64,500 launch directions over all 16
    transmitters), the GPU's logged set of (bounce, receiver) and (bounce,
    edge) equals the oracle's."""
    rows = city_run["captures"]
    assert (rows[:, 3] == 0).sum() >= 200 and (rows[:, 3] == 1).sum() >= 200, np.bincount(rows[:, 3])
    tot = 0
    for t in range(city_run["sc"].n_tx):
        for ids, res in ((city_run["ids"][t], city_run["traces"][t]), (city_run["cov_ids"], city_run["cov_traces"][t])):
            n, bad = P.compare_captures(rows, t, ids, res, strict=False)
            assert not bad, (t, bad[:5])
            tot += n
    assert tot >= 60000


def test_capture_log_marks_and_errors():
    """Marks persist until cleared, a cleared context logs nothing, and a
    direction outside [0, rays_per_tx) is refused."""
    from paper_2303_10521_amd.tracer import EmrtError

    w = city.workload("toy")
    sc = w.scene
    tr = _tracer(sc, w)
    fr = sc.frame(0.0)
    tr.set_frame(fr)
    with pytest.raises(EmrtError):
        tr.debug_select_rays(0, [w.rays_per_tx])
    ids = np.arange(0, w.rays_per_tx, 3, dtype=np.int32)
    tr.debug_select_rays(0, ids)
    tr.step(True)
    a = tr.debug_ray_captures()
    tr.step(True)  # same frame, same marks: the same log
    b = tr.debug_ray_captures()
    assert len(a) > 0 and sorted(map(tuple, a)) == sorted(map(tuple, b))
    res = O.trace(O.OracleScene(sc), O.OracleScene(sc).geometry(fr.obj_xform), fr.tx_pos[0], w.rays_per_tx, ids,
                  w.max_reflections, fr.rx_pos, 1.0, 0, True)
    n, bad = P.compare_captures(a, 0, ids, res)
    assert n >= 0.9 * len(ids) and not bad
    tr.debug_select_rays(0, [])
    tr.step(True)
    assert len(tr.debug_ray_captures()) == 0
    tr.close()


def test_city_discovery_covers_oracle_subset(city_run):
    """Specular keys that the oracle's rays capture robustly on a launch
    subset (every 256th direction of every transmitter, 62,500 rays; a key is
    caught by a few rays of the full 1M-ray lattice) and validates
    unambiguously are in the GPU's path set; so are the unambiguous
    diffraction keys of edges those rays light robustly (a sample of them)."""
    os_, g, fr, w = city_run["os"], city_run["g"], city_run["fr"], city_run["w"]
    gset = P.keyset(city_run["paths"]["key"])
    spec, diff = {}, {}
    for t in range(city_run["sc"].n_tx):
        res = city_run["cov_traces"][t]
        for k, rob in O.spec_keys(os_, res, t).items():
            spec[k] = spec.get(k, False) or rob
        for k, rob in O.diffraction_candidates(os_, g, t, O.illuminated_edges(res), fr.rx_pos,
                                               w.diff_max_leg).items():
            diff[k] = diff.get(k, False) or rob
    ks = np.array([k for k, r in spec.items() if r], np.int32).reshape(-1, 9)
    valid, amb, _, _ = O.validate(os_, g, ks, fr.tx_pos, fr.rx_pos, w.diff_max_leg)
    want = P.keyset(ks[valid & ~amb])
    assert len(want) > 100
    assert want <= gset, sorted(want - gset)[:5]
    kd = np.array([k for k, r in diff.items() if r], np.int32).reshape(-1, 9)
    rng = np.random.default_rng(11)
    kd = kd[rng.choice(len(kd), min(1500, len(kd)), replace=False)]
    valid, amb, _, _ = O.validate(os_, g, kd, fr.tx_pos, fr.rx_pos, w.diff_max_leg)
    want_d = P.keyset(kd[valid & ~amb])
    assert len(want_d) > 20
    assert want_d <= gset, sorted(want_d - gset)[:5]


def test_city_paths_exact_in_oracle(city_run):
    """Sampled GPU paths of every type validate in the oracle with the same
    triangles; gain and Doppler at both carriers, delay and the departure /
    arrival angles agree."""
    os_, g, fr, w = city_run["os"], city_run["g"], city_run["fr"], city_run["w"]
    p = city_run["paths"]
    keys = p["key"]
    rng = np.random.default_rng(3)
    pick = np.concatenate([rng.choice(np.nonzero(keys[:, 2] == t)[0], min(300, int((keys[:, 2] == t).sum())),
                                      replace=False) for t in (0, 1, 2)])
    valid, amb, tri, pts = O.validate(os_, g, keys[pick], fr.tx_pos, fr.rx_pos, w.diff_max_leg)
    assert np.all(valid | amb)
    ok = valid & ~amb
    assert ok.sum() > 0.95 * len(pick)
    a, tau, fd, aod, aoa = O.evaluate(os_, g, keys[pick][ok], pts[ok], fr, w.freqs_hz)
    assert a.shape[1] == 2
    assert np.all(np.abs(p["a"][pick][ok] - a) <= 1e-8 * np.abs(a))
    assert np.all(np.abs(p["tau"][pick][ok] - tau) <= P.TAU_REL * tau)
    assert np.all(np.abs(p["fd"][pick][ok] - fd) <= P.FD_ABS)
    assert P.compare_angles(p["angles"][pick][ok], aod, aoa) <= 1e-6
    spec = keys[pick][ok][:, 2] == 1
    assert np.array_equal(p["tri_ids"][pick][ok][spec], tri[ok][spec])


def test_city_channel_sums_both_carriers(city_run):
    """Per-link sums at 3.5 and 28 GHz (power, delay and Doppler statistics)
    over every path of about 200 sampled links equal the oracle's sums over
    the same keys."""
    os_, g, fr, w, sc = city_run["os"], city_run["g"], city_run["fr"], city_run["w"], city_run["sc"]
    p, ch = city_run["paths"], city_run["ch"]
    link = p["key"][:, 0].astype(np.int64) * sc.n_rx + p["key"][:, 1]
    listed = np.bincount(link, minlength=sc.n_tx * sc.n_rx)
    full = np.nonzero((ch["n_paths"] > 1) & (listed == ch["n_paths"]))[0]  # multipath links, none truncated
    rng = np.random.default_rng(8)
    links = rng.choice(full, min(220, len(full)), replace=False)
    sel = np.isin(link, links)
    keys = p["key"][sel]
    valid, amb, tri, pts = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos, w.diff_max_leg)
    assert np.all(valid | amb)
    a, tau, fd, _, _ = O.evaluate(os_, g, keys, pts, fr, w.freqs_hz)
    ref = O.reduce_links(keys, a, tau, fd, sc.n_tx, sc.n_rx)
    amb_links = set(link[sel][amb].tolist())
    check = np.array([L for L in links if L not in amb_links])
    assert len(check) >= 150
    assert not P.channel_ok(ch, ref, check, 100.0)
    assert np.array_equal(ch["n_paths"][check], ref["n_paths"][check])


# -------------------------------------------------------------- edge cases
def test_toy_at_the_most_reflections():
    """K = 5, the most reflections a context takes, on the toy city with
    diffraction and two carriers, compared in full: hit logs bit-exact on
    robust rays, path sets (specular paths of every order up to 5), per-path
    values and triangles, and every link's channels."""
    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    n, freqs = 50_000, [3.5e9, 28e9]
    tr = _tracer(sc, w, max_reflections=5, rays_per_tx=n, diffraction=1, freq_hz=freqs, path_capacity=1 << 16)
    try:
        tr.set_frame(fr)
        tr.step(True)
        assert tr.sync() == 0
        os_ = O.OracleScene(sc)
        ref = O.run_frame(os_, fr, n, 5, freqs, diffraction=True)
        spec = ref.keys[ref.keys[:, 2] == 1]
        assert set(np.unique(spec[:, 3]).tolist()) == {1, 2, 3, 4, 5}
        t0 = ref.traces[0]
        n_rob, mm_rob, _ = P.compare_hitlogs(tr.debug_rays(0, np.arange(n)), t0.hit_tri, t0.robust)
        assert n_rob >= 0.98 * n and mm_rob == 0
        p = tr.flat_paths(cap=256)
        g = P.keyset(p["key"])
        assert P.keyset(ref.keys[~ref.ambiguous & ref.robust]) <= g
        extra = np.array(sorted(g - P.keyset(ref.keys)), np.int32).reshape(-1, 9)
        if len(extra):
            valid, amb, _, _ = O.validate(os_, os_.geometry(fr.obj_xform), extra, fr.tx_pos, fr.rx_pos)
            assert np.all(valid | amb)
        worst = P.compare_path_values(p["key"], p, ref.keys, dict(a=ref.a, tau=ref.tau, fd=ref.fd), len(freqs))
        assert worst["n"] >= 0.95 * len(ref.keys)
        assert worst["a_rel"] <= 1e-8 and worst["tau_rel"] <= P.TAU_REL and worst["fd_abs"] <= P.FD_ABS, worst
        gi = {tuple(int(x) for x in k): i for i, k in enumerate(p["key"])}
        for j in np.nonzero(~ref.ambiguous)[0]:
            i = gi.get(tuple(int(x) for x in ref.keys[j]))
            if i is not None:
                assert np.array_equal(p["tri_ids"][i], ref.tri_ids[j])
        mask = np.ones(sc.n_tx * sc.n_rx, bool)
        for k in g ^ P.keyset(ref.keys):
            mask[k[0] * sc.n_rx + k[1]] = False
        assert mask.mean() >= 0.9
        assert not P.channel_ok(P.gpu_channels_np(tr.channels()), ref.channels, np.nonzero(mask)[0], 100.0)
    finally:
        tr.close()


def test_no_reflections_only_line_of_sight():
    w = city.workload("toy")
    sc = w.scene
    tr = _tracer(sc, w, max_reflections=0, path_capacity=1 << 12)
    fr = sc.frame(0.0)
    tr.set_frame(fr)
    tr.step(True)
    p = tr.flat_paths()
    assert np.all(p["key"][:, 2] == 0)
    ref = O.run_frame(O.OracleScene(sc), fr, w.rays_per_tx, 0, w.freqs_hz)
    assert P.keyset(p["key"]) == P.keyset(ref.keys)
    tr.close()


def test_single_ray_single_receiver_and_truncation():
    sc = city.tiny_ground_wall(wall_x=50.0)
    sc1 = city.with_static_rx(sc, np.array([[30.0, 20.0, 6.0]]))
    from paper_2303_10521_amd import Tracer

    tr = Tracer(sc1, 1, 1, freq_hz=[28e9], max_reflections=2, rays_per_tx=1, path_capacity=64)
    fr = static_frame([[0.0, 0.0, 10.0]], [[30.0, 20.0, 6.0]])
    tr.set_frame(fr)
    tr.step(True)
    p = tr.flat_paths()
    # a single launch direction (reception sphere 3.5x the path length): same keys as the oracle
    ref = O.run_frame(O.OracleScene(sc1), fr, 1, 2, [28e9])
    assert P.keyset(p["key"]) == P.keyset(ref.keys)
    assert (0, 0, 0, 0, -1, -1, -1, -1, -1) in P.keyset(p["key"])  # line of sight is always tested
    # dense launch: four paths; a path-list capacity of 2 reports truncation
    tr2 = Tracer(sc1, 1, 1, freq_hz=[28e9], max_reflections=2, rays_per_tx=40000, path_capacity=64)
    tr2.set_frame(fr)
    tr2.step(True)
    full = tr2.paths(cap=8)
    assert int(full["count"][0]) == 4 and not full["truncated"]
    cut = tr2.paths(cap=2)
    assert int(cut["count"][0]) == 2 and cut["truncated"]
    ch = tr2.channels()
    assert int(ch["n_paths"][0]) == 4  # sums always use every path
    tr.close()
    tr2.close()


def test_maximum_transmitter_count():
    """4095 transmitters, the most the key references hold (12 bits in a
    diffraction reference), and four carriers, the most a context takes:
    hit logs of the first and last transmitter bit-exact on robust rays, the
    same path sets as the oracle on every link (line of sight, reflections
    and diffraction from every transmitter), per-path values and channels at
    every carrier within tolerance; 4096 transmitters are refused."""
    from paper_2303_10521_amd import Tracer
    from paper_2303_10521_amd.tracer import EmrtError

    sc = city.tiny_box_ground(refl=(0.0, 0.0))
    rng = np.random.default_rng(4095)
    n_tx, n = 4095, 128
    ang, rad = rng.uniform(0, 2 * np.pi, n_tx), rng.uniform(60.0, 300.0, n_tx)
    tx = np.stack([20 + rad * np.cos(ang), 20 + rad * np.sin(ang), rng.uniform(1.5, 45.0, n_tx)], 1)
    rx = np.array([[x, y, 1.5] for x in (-25.0, 70.0) for y in (-30.0, 80.0)] + [[20.0, -60.0, 12.0], [90.0, 20.0, 3.0]])
    sc1 = city.with_static_rx(sc, rx)
    fr = static_frame(tx, rx)
    freqs = [0.9e9, 3.5e9, 28e9, 60e9]
    tr = Tracer(sc1, n_tx, len(rx), freq_hz=freqs, max_reflections=2, rays_per_tx=n, diffraction=1,
                path_capacity=1 << 18)
    try:
        tr.set_frame(fr)
        tr.step(True)
        assert tr.sync() == 0
        os_ = O.OracleScene(sc1)
        ref = O.run_frame(os_, fr, n, 2, freqs, diffraction=1)
        assert ref.keys[:, 0].max() == n_tx - 1 and np.any(ref.keys[ref.keys[:, 0] == n_tx - 1, 2] == 2)
        for t in (0, n_tx - 1):
            tref = ref.traces[t]
            n_rob, mm_rob, _ = P.compare_hitlogs(tr.debug_rays(t, np.arange(n)), tref.hit_tri, tref.robust)
            assert n_rob > 0 and mm_rob == 0, t
        p = tr.flat_paths()
        g = P.keyset(p["key"])
        assert P.keyset(ref.keys[~ref.ambiguous & ref.robust]) <= g
        extra = np.array(sorted(g - P.keyset(ref.keys)), np.int32).reshape(-1, 9)
        if len(extra):
            valid, amb, _, _ = O.validate(os_, os_.geometry(fr.obj_xform), extra, fr.tx_pos, fr.rx_pos)
            assert np.all(valid | amb)
        worst = P.compare_path_values(p["key"], p, ref.keys, dict(a=ref.a, tau=ref.tau, fd=ref.fd), len(freqs))
        assert worst["n"] >= 0.99 * len(ref.keys)
        assert worst["a_rel"] <= 1e-8 and worst["tau_rel"] <= P.TAU_REL and worst["fd_abs"] <= P.FD_ABS, worst
        links = np.arange(n_tx * len(rx))
        assert not P.channel_ok(P.gpu_channels_np(tr.channels()), ref.channels, links, 100.0)
    finally:
        tr.close()
    with pytest.raises(EmrtError) as e:
        Tracer(sc1, n_tx + 1, len(rx), rays_per_tx=n)
    assert e.value.status == -5  # EMRT_E_UNSUPPORTED


def test_error_paths_on_device():
    from paper_2303_10521_amd import Tracer
    from paper_2303_10521_amd.tracer import EmrtError

    w = city.workload("district")
    sc = w.scene
    tr = Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=[28e9], max_reflections=2, rays_per_tx=20000, diffraction=0,
                path_capacity=8)
    fr = sc.frame(0.0)
    tr.set_frame(fr)
    tr.step(True)
    assert tr.sync() == 2  # 8 candidate slots: EMRT_W_CACHE_FULL (a warning, returned not raised)
    bad = sc.frame(0.0)
    bad.obj_xform = bad.obj_xform.copy()
    bad.obj_xform[0, 0, 3] = np.nan
    tr2 = Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=[28e9], max_reflections=1, rays_per_tx=1000, path_capacity=1 << 16)
    tr2.set_frame(bad)
    tr2.step(True)
    with pytest.raises(EmrtError) as e:
        tr2.sync()
    assert e.value.status == -6
    sc_bad = city.workload("toy").scene
    sc_bad.tris = sc_bad.tris.copy()
    sc_bad.tris[3, 1] = len(sc_bad.verts) + 5
    with pytest.raises(EmrtError) as e:
        Tracer(sc_bad, 1, sc_bad.n_rx, rays_per_tx=100)
    assert e.value.status == -1
    tr.close()
    tr2.close()
