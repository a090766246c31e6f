"""Pins of the oracle's receiver-side (backward) launch (Section II-A).

A launch from a receiver with spheres around the transmitters must propose
the same paths as a launch from the transmitters, reversed: reciprocity of
the exact path set.  Pinned against:

* brute-force enumeration on the toy city: every face sequence of order <= 2
  that the image method validates outside its margin is found from the
  receivers' side, and nothing else is;
* the street canyon: exactly the 1 + 2K image paths, the same keys as the
  transmitter-side launch;
* a box building: the corner diffraction round the building found from both
  sides.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import city
from tests.oracle_util import key_set, spec_key, static_frame

F28 = 28e9


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


def test_backward_launch_finds_every_valid_sequence_toy_city():
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr = sc.frame(0.0)
    g = os_.geometry(fr.obj_xform)
    sel = list(range(len(fr.rx_pos)))
    res = O.run_frame(os_, fr, 400000, 2, [F28], want_robust=False, rx_sources=sel)
    F = os_.F
    seqs = [[f] for f in range(F)] + [[f, h] for f in range(F) for h in range(F) if f != h]
    keys = np.array([spec_key(0, r, s) for r in sel for s in seqs], np.int32)
    valid, amb, _, _ = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos)
    brute = key_set(keys[valid & ~amb])
    spec = res.keys[res.keys[:, 2] == 1]
    assert set(int(r) for r in spec[:, 1]) <= set(sel)
    found = key_set(spec)
    assert found <= key_set(keys[valid])
    assert len(brute) > 30
    assert not (brute - found), sorted(brute - found)


@pytest.mark.parametrize("K", [2, 3])
def test_backward_launch_canyon_equals_forward(K):
    gap = 20.0
    sc = city.tiny_canyon(gap=gap)
    os_ = O.OracleScene(sc)
    fr = static_frame([[0.0, 2.0, 0.0]], [[90.0, -5.0, 3.0]])
    fwd = O.run_frame(os_, fr, 60000, K, [F28])
    bwd = O.run_frame(os_, fr, 60000, K, [F28], rx_sources=[0])
    assert len(bwd.keys) == 1 + 2 * K
    assert key_set(bwd.keys) == key_set(fwd.keys)
    np.testing.assert_allclose(bwd.channels["H"], fwd.channels["H"], rtol=1e-14)


def test_backward_launch_corner_diffraction():
    sc = city.tiny_wedge()
    os_ = O.OracleScene(sc)
    fr = static_frame([[-50.0, 20.0, 10.0]], [[20.0, 70.0, 1.5]])
    fwd = O.run_frame(os_, fr, 40000, 2, [F28], diffraction=True)
    bwd = O.run_frame(os_, fr, 40000, 2, [F28], diffraction=True, rx_sources=[0])
    df = {k for k in key_set(fwd.keys) if k[2] == 2}
    db = {k for k in key_set(bwd.keys) if k[2] == 2}
    assert df and df == db
