"""Pins of the oracle's dual-number gradient (``oracle/dual.py``).

The dual-number evaluation rebuilds every path from the transmitter in plain
Python and carries derivatives beside the values.  It is pinned against:

* the C oracle's values: amplitudes at both carriers and unfolded lengths of
  paths of all five types (line of sight, specular up to order 5, wedge
  diffraction, reflection then diffraction, diffraction then reflection), on
  Fresnel materials, so a slip in the value arithmetic of either side shows;
* Fermat / Keller: the unfolded length is stationary in the interaction
  points, so dL/dp_tx = -k_0 (the first leg's direction) for every type, and
  the length does not depend on the dipole orientation;
* the central differences of ``grad_fd`` over the same keys (position,
  orientation of a dipole, complex permittivities) on scenes with all path
  types: two methods that share only the C value code agree to the
  differences' truncation error.
The closed-form gradients (line of sight, normal-incidence permittivity,
dipole orientation, linearity of the loss) run over both methods in
``test_oracle_grad_pins.py``.
"""
import numpy as np
import pytest

from oracle import dual as D
from oracle import oracle as O
from synth import city
from tests.oracle_util import static_frame

FREQS = [3.5e9, 28e9]


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


def _combined_keys(os_, g, fr):
    """All (face, edge) pairs of both orders that validate outside the margin."""
    keys = []
    for f in range(os_.F):
        for e in range(os_.E):
            keys.append([0, 0, 3, 2, f, e, -1, -1, -1])
            keys.append([0, 0, 4, 2, e, f, -1, -1, -1])
    keys = np.array(keys, np.int32)
    out = []
    for rx in range(len(fr.rx_pos)):
        k = keys.copy()
        k[:, 1] = rx
        valid, amb, _, _ = O.validate(os_, g, k, fr.tx_pos, fr.rx_pos)
        out.append(k[valid & ~amb])
    return np.concatenate(out)


def _box_case():
    """A Fresnel box on a Fresnel ground, receivers all round it: every path
    type up to order 2, with first-order diffraction and both combined
    orders."""
    sc = city.tiny_box_ground(refl=(0.0, 0.0))
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[-30.0, 20.0, 2.0]])
    rx = np.array([[x, y, z] for x in (-20.0, 60.0) for y in (-20.0, 75.0) for z in (1.5, 25.0)])
    fr = static_frame(tx, rx, tx_orient=[[0.8, -0.4]])
    ref = O.run_frame(os_, fr, 20000, 2, FREQS, diffraction=1)
    keys = np.concatenate([ref.keys[~ref.ambiguous], _combined_keys(os_, g, fr)])
    return os_, g, fr, keys


def _toy_case():
    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    fr.tx_orient = np.array([[0.6, 0.4]])
    os_ = O.OracleScene(sc)
    g = os_.geometry(fr.obj_xform)
    ref = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, FREQS, diffraction=1)
    return os_, g, fr, ref.keys[~ref.ambiguous]


@pytest.fixture(scope="module", params=["box", "toy"])
def case(request):
    return _box_case() if request.param == "box" else _toy_case()


def test_cases_cover_every_path_type():
    for build, want in ((_box_case, {0, 1, 2, 3, 4}), (_toy_case, {0, 1, 2})):
        keys = build()[3]
        assert set(np.unique(keys[:, 2]).tolist()) == want


@pytest.mark.parametrize("ant_mode", [0, 1])
def test_values_equal_the_c_oracle(case, ant_mode):
    os_, g, fr, keys = case
    a, _, L, _ = D.evaluate_dual(os_, g, fr, keys, FREQS, ant_mode)
    pts = O.image_points(os_, g, keys, fr.tx_pos, fr.rx_pos)
    ac, tau, _, _, _ = O.evaluate(os_, g, keys, pts, fr, FREQS, ant_mode)
    # the phase is taken modulo one wavelength of a length of ~100 m: a few
    # ulps of the length move it by ~1e-11 rad at 28 GHz
    assert np.all(np.abs(a - ac) <= 1e-9 * np.abs(ac)), np.max(np.abs(a - ac) / np.abs(ac))
    assert np.allclose(L, tau * O.C0, rtol=1e-13, atol=0)


def test_length_is_stationary_in_the_points(case):
    """Fermat (specular) and Keller (diffraction): dL/dp_tx = -k_0."""
    os_, g, fr, keys = case
    _, _, _, dL = D.evaluate_dual(os_, g, fr, keys, FREQS[:1], 1)
    pts = O.image_points(os_, g, keys, fr.tx_pos, fr.rx_pos)
    first = np.where((keys[:, 2] == 0)[:, None], fr.rx_pos[keys[:, 1]], pts[:, 0])
    k0 = first - fr.tx_pos[keys[:, 0]]
    k0 /= np.linalg.norm(k0, axis=1, keepdims=True)
    assert np.abs(dL[:, :3] + k0).max() < 1e-12
    assert np.all(dL[:, 3:] == 0)


def _rel_err(got, want):
    got, want = np.atleast_2d(got), np.atleast_2d(want)
    scale = np.maximum(np.abs(want).max(axis=1, keepdims=True), 1e-300)
    return float((np.abs(got - want) / scale).max())


@pytest.mark.parametrize("ant_mode", [0, 1])
def test_dual_numbers_agree_with_central_differences(case, ant_mode):
    os_, g, fr, keys = case
    n_rx = len(fr.rx_pos)
    nl = len(fr.tx_pos) * n_rx
    r = np.random.default_rng(11 + ant_mode)
    GH = r.normal(size=(2, nl)) + 1j * r.normal(size=(2, nl))
    GP = r.normal(size=(2, nl)) * 1e6
    want = O.grad_fd(os_, g, fr, keys, FREQS, GH, GP, n_rx, ant_mode=ant_mode)
    got = D.grad_dual(os_, g, fr, keys, FREQS, GH, GP, n_rx, ant_mode=ant_mode)
    names = ("grad_tx_pos", "grad_eps") + (("grad_tx_orient",) if ant_mode == 1 else ())
    for name in names:
        assert np.abs(want[name]).max() > 0, name
        err = _rel_err(got[name], want[name])
        assert err < 2e-6, (name, err)
    if ant_mode == 0:
        assert np.all(got["grad_tx_orient"] == 0)


def test_a_dropped_chain_rule_term_is_caught():
    """Planted mistake, on the CPU: a square root whose derivative loses its
    factor 1/2 changes the dual gradient well beyond the agreement bar above
    (guards that the comparison can fail)."""
    os_, g, fr, keys = _box_case()
    n_rx = len(fr.rx_pos)
    r = np.random.default_rng(5)
    GH = r.normal(size=(2, n_rx)) + 1j * r.normal(size=(2, n_rx))
    good = D.grad_dual(os_, g, fr, keys, FREQS, GH, None, n_rx)
    orig = D.dsqrt

    def bad_sqrt(x):
        y = orig(x)
        return D.Dual(y.v, y.d * 2.0) if isinstance(y, D.Dual) else y

    D.dsqrt = bad_sqrt
    try:
        bad = D.grad_dual(os_, g, fr, keys, FREQS, GH, None, n_rx)
    finally:
        D.dsqrt = orig
    assert _rel_err(bad["grad_tx_pos"], good["grad_tx_pos"]) > 1e-2
