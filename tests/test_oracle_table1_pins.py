"""Pins of the oracle's constant reflection coefficients (Section IV, Table I)
and of the Table III street scenario.

Table I gives its wall and metal surfaces a reflection coefficient alone
(0.8 and 0.9).  The oracle reads it as a coefficient of that magnitude at
every angle and for both polarisations, with a perfect conductor's signs.
Pinned here against:

* the two-ray ground model with the image of a vertical dipole over a
  conductor scaled by g (vertical polarisation: the parallel coefficient +g);
* the street canyon between two walls, where every path keeps its vertical
  polarisation, so an n-bounce path carries (-g)^n (the perpendicular
  coefficient) and H is a sum over the unfolded images;
* the conductor limit: with g = 1 every channel, with diffraction at a
  wedge too, equals the one of a material whose permittivity tends to
  infinity (here eps = 1 - 1e14 j), through the Fresnel forms;
* Table III: on the street scenario the mean Doppler shift and the RMS
  Doppler spread scale by exactly 5 from 10 to 50 m/s (the paper's rows are
  x5), the path set and the power do not change, and the mean shift is low
  abeam (10 m, line of sight perpendicular to the motion) and large at 300 m.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import city
from tests.oracle_util import C0, key_set, spec_key, static_frame

F30 = 30e9


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


def _with_refl(sc, refl):
    return dataclasses.replace(sc, material_refl=np.asarray(refl, np.float64))


def _run(sc, tx, rx, N, K, diffraction=False, freqs=(F30,)):
    os_ = O.OracleScene(sc)
    fr = static_frame(tx, rx)
    return O.run_frame(os_, fr, N, K, list(freqs), diffraction=diffraction)


@pytest.mark.parametrize("g", [0.8, 0.9, 1.0])
def test_two_ray_ground_with_a_constant_coefficient(g):
    sc = _with_refl(city.tiny_ground(), [g])
    tx = np.array([[0.0, 0.0, 10.0]])
    rx = np.array([[80.0, 30.0, 1.5]])
    res = _run(sc, tx, rx, 20000, 2)
    assert key_set(res.keys) == {tuple(spec_key(0, 0, [])), tuple(spec_key(0, 0, [0]))}
    lam = C0 / F30
    k = 2 * math.pi / lam
    d = float(np.linalg.norm(rx - tx))
    r = float(np.linalg.norm(rx - tx * np.array([1, 1, -1])))
    h = lam / (4 * math.pi) * (np.exp(-1j * k * d) / d + g * np.exp(-1j * k * r) / r)
    assert abs(res.channels["H"][0, 0] - h) < 1e-9 * abs(h)


@pytest.mark.parametrize("g", [0.8, 0.9])
def test_canyon_paths_carry_minus_g_per_bounce(g):
    gap, K = 20.0, 3
    sc = _with_refl(city.tiny_canyon(gap=gap), [g])
    tx = np.array([[0.0, 2.0, 0.0]])
    rx = np.array([[90.0, -5.0, 0.0]])  # same height: horizontal rays, vertical E
    res = _run(sc, tx, rx, 60000, K)
    assert len(res.keys) == 1 + 2 * K
    lam = C0 / F30
    k = 2 * math.pi / lam
    h = 0j
    for first in (gap / 2, -gap / 2):
        img = tx[0].copy()
        wall = first
        for n in range(1, K + 1):
            img[1] = 2 * wall - img[1]
            L = float(np.linalg.norm(rx[0] - img))
            h += (-g) ** n * np.exp(-1j * k * L) / L
            wall = -wall
    d = float(np.linalg.norm(rx[0] - tx[0]))
    h = lam / (4 * math.pi) * (h + np.exp(-1j * k * d) / d)
    assert abs(res.channels["H"][0, 0] - h) < 1e-9 * abs(h)


def test_unit_coefficient_is_the_conductor_limit_with_diffraction():
    conductor = 1.0 - 1.0e14j
    for base, tx, rx in [
        (city.tiny_ground_wall(), [[0.0, 0.0, 10.0]], [[30.0, 25.0, 1.5]]),
        (city.tiny_wedge(), [[-50.0, 20.0, 10.0]], [[20.0, 70.0, 1.5]]),  # round the corner
    ]:
        M = len(base.materials)
        a = _run(_with_refl(base, np.ones(M)), np.array(tx), np.array(rx), 40000, 2, diffraction=True)
        b = _run(dataclasses.replace(base, materials=np.full(M, conductor)), np.array(tx), np.array(rx), 40000, 2,
                 diffraction=True)
        assert key_set(a.keys) == key_set(b.keys)
        assert len(a.keys) >= 2
        h1, h2 = a.channels["H"][0, 0], b.channels["H"][0, 0]
        assert abs(h1 - h2) < 1e-5 * abs(h2)
    # the diffracted path alone, too
    kinds = {int(k[2]) for k in np.asarray(a.keys).reshape(-1, 9)}
    assert 2 in kinds


def test_table3_speed_structure_on_the_street_scenario():
    stats = {}
    for d in (10.0, 300.0):
        runs = {}
        for v in (10.0, 50.0):
            w = city.table3_street(d, v)
            assert w.freqs_hz == (30e9,)
            assert list(w.scene.material_refl) == [city.REFL_WALL, city.REFL_METAL]
            fr = w.scene.frame(0.0)
            assert abs(np.linalg.norm(fr.rx_pos[0] - fr.tx_pos[0]) - d) < 1e-9 * d
            os_ = O.OracleScene(w.scene)
            runs[v] = O.run_frame(os_, fr, 100_000, w.max_reflections, list(w.freqs_hz), diffraction=True)
        r1, r5 = runs[10.0], runs[50.0]
        assert key_set(r1.keys) == key_set(r5.keys)
        assert len(r1.keys) > 10
        np.testing.assert_allclose(r5.fd, 5.0 * r1.fd, rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(r5.channels["P_coh"], r1.channels["P_coh"], rtol=1e-12)
        for name in ("fd_mean", "fd_rms"):
            np.testing.assert_allclose(r5.channels[name], 5.0 * r1.channels[name], rtol=1e-9, atol=1e-12)
        stats[d] = (float(r1.channels["fd_mean"][0, 0]), float(r1.channels["fd_rms"][0, 0]))
    # abeam the line of sight carries no Doppler; at 300 m it is nearly v / lambda
    v_over_lam = 10.0 * 30e9 / C0
    assert abs(stats[10.0][0]) < 0.01 * v_over_lam
    assert 0.9 * v_over_lam < stats[300.0][0] <= v_over_lam
