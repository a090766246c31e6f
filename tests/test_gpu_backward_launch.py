"""Receiver-side (backward) discovery on the GPU (emrt_step_rx) against the
oracle's receiver-side launch, through the C ABI.

* Toy city, first step launched from four receivers (K = 3, diffraction on):
  path sets, per-path values and every link's channels against the oracle.
* Toy city, a transmitter-side discovery frame, then a later frame that
  rediscovers from three receivers with the cache revalidated for all links:
  the same comparison, each side carrying its own cache.
* Reciprocity: in the street canyon the receiver-side launch yields exactly
  the transmitter-side path set and the same channel.
* The most receivers one step launches from (1024), against the oracle.
* Argument and state errors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402
from tests import parity as P  # noqa: E402
from tests.oracle_util import static_frame  # noqa: E402

pytestmark = pytest.mark.gpu

N_RX = 50_000


def _tracer(sc, n_tx, n_rx, rays_per_tx, K, diffraction, cap=1 << 16):
    from paper_2303_10521_amd import Tracer

    return Tracer(sc, n_tx, n_rx, freq_hz=[28e9], max_reflections=K, rays_per_tx=rays_per_tx,
                  diffraction=int(diffraction), path_capacity=cap)


def _compare(gpu_paths, gpu_ch, ref, os_, fr, n_links):
    g = P.keyset(gpu_paths["key"])
    assert P.keyset(ref.keys[~ref.ambiguous & ref.robust]) <= g
    extra = np.array(sorted(g - P.keyset(ref.keys)), np.int32).reshape(-1, 9)
    if len(extra):
        valid, amb, _, _ = O.validate(os_, os_.geometry(fr.obj_xform), extra, fr.tx_pos, fr.rx_pos)
        assert np.all(valid | amb)
    assert len(extra) <= max(1, len(g) // 50)
    gi = {tuple(int(x) for x in k): i for i, k in enumerate(gpu_paths["key"])}
    n = 0
    for j, k in enumerate(ref.keys):
        i = gi.get(tuple(int(x) for x in k))
        if i is None:
            continue
        n += 1
        assert abs(gpu_paths["a"][i, 0] - ref.a[j, 0]) <= 1e-8 * abs(ref.a[j, 0])
        assert abs(gpu_paths["tau"][i] - ref.tau[j]) <= P.TAU_REL * ref.tau[j]
        assert abs(gpu_paths["fd"][i, 0] - ref.fd[j, 0]) <= P.FD_ABS
    assert n >= 0.95 * len(ref.keys)
    # every link: those of launched receivers and those only revalidated
    mask = np.ones(n_links, bool)
    for k in set(g) ^ P.keyset(ref.keys):
        mask[k[0] * len(fr.rx_pos) + k[1]] = False
    assert mask.mean() >= 0.9
    assert not P.channel_ok(gpu_ch, ref.channels, np.nonzero(mask)[0], 100.0)


def test_toy_first_step_from_receivers():
    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    sel = [1, 6, 11, 15]
    tr = _tracer(sc, sc.n_tx, sc.n_rx, len(sel) * N_RX, 3, True)
    tr.set_frame(fr)
    tr.step_rx(sel, N_RX)
    assert tr.sync() == 0
    p = tr.flat_paths(cap=256)
    os_ = O.OracleScene(sc)
    ref = O.run_frame(os_, fr, N_RX, 3, [28e9], diffraction=True, rx_sources=sel)
    # only the launched receivers gain reflected or diffracted paths
    assert set(int(r) for r in p["key"][p["key"][:, 2] != 0, 1]) <= set(sel)
    assert (p["key"][:, 2] == 2).any() and (p["key"][:, 2] == 1).any()
    _compare(p, P.gpu_channels_np(tr.channels()), ref, os_, fr, sc.n_tx * sc.n_rx)
    tr.close()


def test_toy_rediscovery_after_a_cached_schedule():
    w = city.workload("toy")
    sc = w.scene
    f0, f1 = sc.frame(0.0), sc.frame(0.0)
    f1.rx_pos = f1.rx_pos + np.array([1.5, -0.75, 0.0])  # every receiver moved
    sel = [2, 9, 13]
    tr = _tracer(sc, sc.n_tx, sc.n_rx, w.rays_per_tx, 3, True)
    tr.set_frame(f0, 0)
    tr.step(True)
    tr.set_frame(f1, 1)
    tr.step_rx(sel, w.rays_per_tx // len(sel))
    assert tr.sync() == 0
    os_ = O.OracleScene(sc)
    r0 = O.run_frame(os_, f0, w.rays_per_tx, 3, [28e9], diffraction=True)
    r1 = O.run_frame(os_, f1, w.rays_per_tx // len(sel), 3, [28e9], diffraction=True, rx_sources=sel,
                     cache=O.cache_of(r0))
    _compare(tr.flat_paths(cap=256), P.gpu_channels_np(tr.channels()), r1, os_, f1, sc.n_tx * sc.n_rx)
    tr.close()


@pytest.mark.parametrize("K", [2, 3])
def test_canyon_reciprocity(K):
    sc = city.with_static_rx(city.tiny_canyon(gap=20.0), np.array([[90.0, -5.0, 3.0]]))
    fr = static_frame([[0.0, 2.0, 0.0]], [[90.0, -5.0, 3.0]])
    a = _tracer(sc, 1, 1, 60000, K, False, cap=256)
    a.set_frame(fr)
    a.step(True)
    b = _tracer(sc, 1, 1, 60000, K, False, cap=256)
    b.set_frame(fr)
    b.step_rx([0], 60000)
    assert a.sync() == 0 and b.sync() == 0
    pa, pb = a.flat_paths(), b.flat_paths()
    assert len(pa["key"]) == 1 + 2 * K
    assert np.array_equal(pa["key"], pb["key"])
    assert np.array_equal(pa["a"], pb["a"])
    assert torch.equal(a.channels()["H"], b.channels()["H"])
    a.close()
    b.close()


def test_launch_from_the_most_receivers():
    """1024 receivers launching at once, the most one receiver-side step
    takes (64 rays each, K = 2, diffraction on): path sets, per-path values
    and channels against the oracle's receiver-side launch; 1025 are
    refused."""
    from paper_2303_10521_amd.tracer import EmrtError

    sc = city.tiny_box_ground(refl=(0.0, 0.0))
    rng = np.random.default_rng(1024)
    n_rx, per = 1024, 64
    ang, rad = rng.uniform(0, 2 * np.pi, n_rx), rng.uniform(45.0, 250.0, n_rx)
    rx = np.stack([20 + rad * np.cos(ang), 20 + rad * np.sin(ang), rng.uniform(1.5, 20.0, n_rx)], 1)
    tx = np.array([[-40.0, 20.0, 25.0], [80.0, 70.0, 10.0]])
    sc1 = city.with_static_rx(sc, rx)
    fr = static_frame(tx, rx)
    tr = _tracer(sc1, len(tx), n_rx, n_rx * per // len(tx), 2, True)
    try:
        tr.set_frame(fr)
        tr.step_rx(list(range(n_rx)), per)
        assert tr.sync() == 0
        p = tr.flat_paths(cap=64)
        os_ = O.OracleScene(sc1)
        ref = O.run_frame(os_, fr, per, 2, [28e9], diffraction=True, rx_sources=list(range(n_rx)))
        assert set(np.unique(ref.keys[:, 2]).tolist()) == {0, 1, 2}
        _compare(p, P.gpu_channels_np(tr.channels()), ref, os_, fr, len(tx) * n_rx)
        with pytest.raises(EmrtError):
            tr.step_rx([0] * (n_rx + 1), 1)
    finally:
        tr.close()


def test_receiver_launch_errors():
    from paper_2303_10521_amd.tracer import EmrtError

    w = city.workload("toy")
    sc = w.scene
    tr = _tracer(sc, sc.n_tx, sc.n_rx, w.rays_per_tx, 3, False)
    tr.set_frame(sc.frame(0.0))
    for ids, rays in (([sc.n_rx], 100), ([-1], 100), ([0, 1], w.rays_per_tx), ([], 100), ([0], 0)):
        with pytest.raises(EmrtError):
            tr.step_rx(ids, rays)
    tr.step_rx([0, 0, 3], 1000)  # repeats are allowed
    assert tr.sync() == 0
    with pytest.raises(EmrtError):
        tr.debug_rays(0, np.arange(4))  # the hit log holds a receiver-side launch
    tr.step(True)
    assert tr.debug_rays(0, np.arange(4)).shape == (4, 4)
    tr.close()
