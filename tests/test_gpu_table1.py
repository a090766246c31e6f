"""Table I's constant reflection coefficients and Table III's street scenario
on the GPU, against the oracle, through the C ABI
(emrt_set_reflection_coefficients).

* The four Table III rows (10 / 50 m/s, 10 / 300 m, 30 GHz, walls and ground
  0.8, the metal vehicle 0.9, first-order diffraction, K = 4): path sets,
  per-path values and channels against the oracle at the tolerances of
  tests/parity.py.
* The speed structure on the GPU's own outputs: the same paths at both speeds,
  every Doppler shift and both Doppler statistics x5, powers unchanged.
* The adjoint with one constant material among Fresnel ones: its
  permittivity gradient is exactly zero, the others match the oracle's central
  differences.
* Argument errors.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402
from tests import parity as P  # noqa: E402

pytestmark = pytest.mark.gpu

ROWS = [(10.0, 10.0), (10.0, 300.0), (50.0, 10.0), (50.0, 300.0)]  # (m/s, m)
N = 100_000


@pytest.fixture(scope="module")
def rows():
    from paper_2303_10521_amd import Tracer

    out = {}
    for v, d in ROWS:
        w = city.table3_street(d, v, rays_per_tx=N)
        sc = w.scene
        fr = sc.frame(0.0)
        tr = Tracer(sc, 1, 1, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=N,
                    diffraction=1, diff_max_leg_m=w.diff_max_leg, path_capacity=1 << 16)
        tr.set_frame(fr)
        tr.step(True)
        assert tr.sync() == 0
        os_ = O.OracleScene(sc)
        ref = O.run_frame(os_, fr, N, w.max_reflections, list(w.freqs_hz), diffraction=True,
                          diff_max_leg=w.diff_max_leg)
        out[(v, d)] = dict(os=os_, fr=fr, paths=tr.flat_paths(cap=256), ch=P.gpu_channels_np(tr.channels()),
                           ref=ref)
        tr.close()
    return out


@pytest.mark.parametrize("row", ROWS)
def test_table3_rows_match_the_oracle(rows, row):
    r = rows[row]
    ref, p = r["ref"], r["paths"]
    g = P.keyset(p["key"])
    assert P.keyset(ref.keys[~ref.ambiguous & ref.robust]) <= g
    extra = np.array(sorted(g - P.keyset(ref.keys)), np.int32).reshape(-1, 9)
    if len(extra):
        valid, amb, _, _ = O.validate(r["os"], r["os"].geometry(r["fr"].obj_xform), extra, r["fr"].tx_pos,
                                      r["fr"].rx_pos)
        assert np.all(valid | amb)
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
    assert n >= 0.95 * len(ref.keys) and n > 10
    assert not P.channel_ok(r["ch"], ref.channels, np.arange(1), 100.0)


@pytest.mark.parametrize("d", [10.0, 300.0])
def test_table3_speed_structure_on_the_gpu(rows, d):
    a, b = rows[(10.0, d)], rows[(50.0, d)]
    assert np.array_equal(a["paths"]["key"], b["paths"]["key"])
    np.testing.assert_allclose(b["paths"]["fd"], 5.0 * a["paths"]["fd"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(b["ch"]["P_coh"], a["ch"]["P_coh"], rtol=1e-12)
    for name in ("fd_mean", "fd_rms"):
        np.testing.assert_allclose(b["ch"][name], 5.0 * a["ch"][name], rtol=1e-9, atol=1e-12)


def test_constant_material_adjoint():
    """Toy city with its facade material (index 1) at a constant 0.8 and the
    ground and metal on Fresnel coefficients."""
    from tests.test_gpu_adjoint import _check, _run

    w = city.workload("toy")
    sc = dataclasses.replace(w.scene, material_refl=np.array([0.0, city.REFL_WALL, 0.0]))
    fr = sc.frame(0.0)
    tr, got, wants, _ = _run(sc, fr, sc.n_tx, sc.n_rx, w.max_reflections, w.rays_per_tx, w.freqs_hz, False, 0, 4)
    assert got["grad_eps"][1] == 0
    assert all(want["grad_eps"][1] == 0 for want in wants.values())
    assert np.abs(got["grad_eps"]).max() > 0
    _check(got, wants, ("grad_tx_pos", "grad_eps"))
    tr.close()


def test_reflection_coefficient_errors():
    from paper_2303_10521_amd import Tracer
    from paper_2303_10521_amd.tracer import EmrtError

    w = city.workload("toy")
    sc = w.scene
    tr = Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections,
                rays_per_tx=w.rays_per_tx, path_capacity=1 << 16)
    M = len(sc.materials)
    for bad in (np.full(M + 1, 0.5), np.array([0.5, 1.5, 0.5][:M]), np.array([0.5, np.nan, 0.5][:M]),
                np.array([-0.1, 0.5, 0.5][:M])):
        with pytest.raises(EmrtError):
            tr.set_reflection_coefficients(bad)
    tr.set_reflection_coefficients(np.full(M, 0.9))
    tr.close()
