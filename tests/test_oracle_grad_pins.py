"""Pins of the oracle's two gradients (central differences over the FP64
oracle, ``grad_fd``, and forward-mode dual numbers, ``dual.grad_dual``; both
with the path topology held fixed) against closed forms.

The gradients are those of a real loss of the per-link channels,
L = sum_{f, link} Re(conj(G_H) H) + G_P P_tx |H|^2, with respect to the
transmitter position, the dipole orientation and the complex permittivity of
each material (PyTorch convention dL/dRe + j dL/dIm).  Each pin is a case
where the derivative has a closed form that does not go through the oracle:

* line of sight: a = lambda/(4 pi d) e^{-j k d}, so da/dp_tx = a (-1/d - j k)
  dd/dp_tx with dd/dp_tx = (p_tx - p_rx)/d;
* normal incidence on the ground: a = -C Gamma_TM(eps) with
  dGamma_TM/deps = 1 / (sqrt(eps) (sqrt(eps) + 1)^2);
* dipole orientation: a is linear in the transmit polarisation vector;
* Fermat / Keller: the unfolded length of a specular or diffracted path is
  stationary in its interaction points, so dL/dp_tx = -k_0 (first leg), which
  fails if the fixed-topology points are wrong.
"""
import numpy as np
import pytest

from oracle import dual as D
from oracle import oracle as O
from synth import city
from tests.oracle_util import C0, spec_key, static_frame

F28 = 28e9
F35 = 3.5e9


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


# both gradient methods take the same arguments and return the same dict
METHODS = pytest.mark.parametrize("grad", [O.grad_fd, D.grad_dual], ids=["central_differences", "dual_numbers"])


def _rng_G(nf, nl, seed=0):
    r = np.random.default_rng(seed)
    return r.normal(size=(nf, nl)) + 1j * r.normal(size=(nf, nl)), r.normal(size=(nf, nl))


def _los_amp(tx, rx, lam):
    d = np.linalg.norm(rx - tx)
    return lam / (4 * np.pi * d) * np.exp(-2j * np.pi * d / lam), d


@METHODS
def test_los_position_gradient_closed_form(grad):
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([3.0, 4.0, 10.0])
    rx = np.array([40.0, -25.0, 1.5])
    fr = static_frame([tx], [rx])
    freqs = [F28, F35]
    GH, GP = _rng_G(2, 1, 1)
    GP = GP * 1e6  # comparable weight of the power term (|a|^2 P_tx ~ 1e-6)
    keys = np.array([spec_key(0, 0, [])])
    got = grad(os_, g, fr, keys, freqs, GH, GP, 1)["grad_tx_pos"][0]
    want = np.zeros(3)
    for fi, f in enumerate(freqs):
        lam = C0 / f
        a, d = _los_amp(tx, rx, lam)
        dd = (tx - rx) / d
        da = a * (-1.0 / d - 2j * np.pi / lam) * dd
        want += (np.conj(GH[fi, 0]) * da).real + GP[fi, 0] * O.P_TX_W * 2 * (np.conj(a) * da).real
    assert np.allclose(got, want, rtol=1e-6, atol=1e-9 * np.abs(want).max())


@METHODS
def test_normal_incidence_permittivity_gradient_closed_form(grad):
    eps = 15.0 - 1.5j
    sc = city.tiny_ground(eps=eps)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    fr = static_frame([[0.0, 0.0, 10.0]], [[0.0, 0.0, 5.0]])
    GH, _ = _rng_G(1, 1, 2)
    keys = np.array([spec_key(0, 0, [0])])
    got = grad(os_, g, fr, keys, [F28], GH, None, 1)["grad_eps"][0]
    lam = C0 / F28
    L = 15.0
    C = lam / (4 * np.pi * L) * np.exp(-2j * np.pi * (L / lam - np.round(L / lam)))
    r = np.sqrt(eps)
    da = -C / (r * (r + 1) ** 2)
    want = GH[0, 0] * np.conj(da)
    assert abs(got - want) <= 1e-6 * abs(want)


@METHODS
def test_dipole_orientation_gradient_closed_form(grad):
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([0.0, 0.0, 30.0])
    rx = np.array([80.0, 35.0, 1.5])
    th, ph = 0.7, 0.3
    fr = static_frame([tx], [rx], tx_orient=[[th, ph]])
    GH, _ = _rng_G(1, 1, 3)
    keys = np.array([spec_key(0, 0, [])])
    got = grad(os_, g, fr, keys, [F28], GH, None, 1, ant_mode=1)["grad_tx_orient"][0]
    lam = C0 / F28
    k = (rx - tx) / np.linalg.norm(rx - tx)
    a0, _ = _los_amp(tx, rx, lam)
    z = np.array([0.0, 0.0, 1.0])
    er = z - (z @ k) * k
    er /= np.linalg.norm(er)
    u_th = np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    u_ph = np.array([-np.sin(th) * np.sin(ph), np.sin(th) * np.cos(ph), 0.0])
    want = []
    for du in (u_th, u_ph):
        de = np.sqrt(1.5) * (du - (du @ k) * k)
        want.append((np.conj(GH[0, 0]) * a0 * (er @ de)).real)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-12)


def _tau(os_, g, fr, keys, tx):
    f2 = O._FrameView(fr, tx_pos=np.array([tx]))
    pts = O.image_points(os_, g, keys, f2.tx_pos, f2.rx_pos)
    _, tau, _, _, _ = O.evaluate(os_, g, keys, pts, f2, [F28])
    return tau, pts


@pytest.mark.parametrize("faces", [[0], [1], [0, 1], [1, 0], [0, 1, 0], [1, 0, 1, 0, 1]])
def test_fermat_specular_length_gradient(faces):
    sc = city.tiny_canyon(gap=20.0)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([-100.0, 1.0, 3.0])
    rx = np.array([150.0, -2.0, 1.0])
    fr = static_frame([tx], [rx])
    keys = np.array([spec_key(0, 0, faces)])
    valid, _, _, _ = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos)
    assert valid[0]
    _, pts = _tau(os_, g, fr, keys, tx)
    k0 = pts[0, 0] - tx
    k0 /= np.linalg.norm(k0)
    h = 1e-3
    grad = np.zeros(3)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        grad[c] = (_tau(os_, g, fr, keys, tx + e)[0][0] - _tau(os_, g, fr, keys, tx - e)[0][0]) / (2 * h) * C0
    assert np.allclose(grad, -k0, atol=1e-7)


def test_keller_diffracted_length_gradient():
    sc = city.tiny_wedge(size=40.0, height=30.0)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([-30.0, 20.0, 40.0])
    rx = np.array([60.0, 70.0, 1.5])
    fr = static_frame([tx], [rx])
    keys = np.array([[0, 0, 2, 1, e, -1, -1, -1, -1] for e in range(os_.E)], np.int32)
    valid, amb, _, _ = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos)
    ok = np.flatnonzero(valid & ~amb)
    assert len(ok) >= 1
    h = 1e-3
    for q in ok:
        kq = keys[q:q + 1]
        _, pts = _tau(os_, g, fr, kq, tx)
        k0 = pts[0, 0] - tx
        k0 /= np.linalg.norm(k0)
        grad = np.zeros(3)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            grad[c] = (_tau(os_, g, fr, kq, tx + e)[0][0] - _tau(os_, g, fr, kq, tx - e)[0][0]) / (2 * h) * C0
        assert np.allclose(grad, -k0, atol=1e-7)


@METHODS
def test_gradient_loss_terms_add(grad):
    """The loss is linear in (G_H, G_P): gradients of the two terms add."""
    sc = city.tiny_ground_wall()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    fr = static_frame([[0.0, 0.0, 10.0]], [[30.0, 20.0, 6.0]])
    keys = np.array([spec_key(0, 0, f) for f in ([], [0], [1], [0, 1])])
    GH, GP = _rng_G(1, 1, 4)
    a = grad(os_, g, fr, keys, [F28], GH, None, 1)
    b = grad(os_, g, fr, keys, [F28], 0 * GH, GP, 1)
    c = grad(os_, g, fr, keys, [F28], GH, GP, 1)
    for name in ("grad_tx_pos", "grad_eps"):
        assert np.allclose(a[name] + b[name], c[name], rtol=1e-6, atol=1e-12)
