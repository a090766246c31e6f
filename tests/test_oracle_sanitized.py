"""The oracle under the address and undefined-behaviour sanitizers (host code).

The C oracle is rebuilt with ``-fsanitize=address,undefined`` and the oracle
pin suites run against that build in a child process (sanitizer runtime
preloaded, any report fatal).  Malformed path keys are also fed straight to
the C routines, past the Python check: they must be counted and rejected,
never indexed (a key with more than five reflections once overran the
construction's point arrays).
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O
from synth import city

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = [
    "tests/test_oracle_pins.py",
    "tests/test_oracle_grad_pins.py",
    "tests/test_oracle_refl_diff_pins.py",
    "tests/test_oracle_backward_pins.py",
    "tests/test_oracle_table1_pins.py",
    "tests/test_oracle_coherence_pins.py",
    "tests/test_oracle_output_pins.py",
]


def _malformed(F, E):
    good = [0, 0, 1, 2, 0, 1, -1, -1, -1]
    rows = [
        [0, 0, 1, 6, 0, 1, 2, 3, 4],       # six reflections (the point arrays hold five)
        [0, 0, 1, 0, -1, -1, -1, -1, -1],  # specular without a face
        [0, 0, 1, 2, 0, F, -1, -1, -1],    # face id out of range
        [0, 0, 1, 1, -7, -1, -1, -1, -1],  # negative face id
        [0, 0, 2, 1, E, -1, -1, -1, -1],   # edge id out of range
        [0, 0, 2, 2, 0, -1, -1, -1, -1],   # diffraction of order 2
        [0, 0, 3, 2, 0, E + 3, -1, -1, -1],  # reflection-diffraction with a bad edge
        [0, 0, 4, 2, 0, F + 1, -1, -1, -1],  # diffraction-reflection with a bad face
        [0, 0, 9, 1, 0, -1, -1, -1, -1],   # unknown type
        [0, 0, 0, 3, -1, -1, -1, -1, -1],  # line of sight with an order
        [5, 0, 0, 0, -1, -1, -1, -1, -1],  # transmitter out of range
        [0, 999, 1, 1, 0, -1, -1, -1, -1],  # receiver out of range
        [0, -1, 0, 0, -1, -1, -1, -1, -1],  # negative receiver
    ]
    return np.array([good] + rows, np.int32), len(rows)


def test_malformed_keys_rejected_in_c():
    """orc_validate / orc_image_points / orc_eval count malformed rows, mark
    them invalid and leave them unindexed; the well-formed row still
    validates.  The Python wrappers raise MalformedKey with the row."""
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr = sc.frame(0.0)
    g = os_.geometry(fr.obj_xform)
    keys, nbad = _malformed(os_.F, os_.E)
    n = len(keys)
    lib = O.lib()
    i32, p = ctypes.c_int32, O._p
    valid = np.full(n, 7, np.uint8)
    amb = np.full(n, 7, np.uint8)
    tri = np.zeros((n, 5), np.int32)
    pts = np.zeros((n, 5, 3))
    tx, rx = O._c(fr.tx_pos, np.float64), O._c(fr.rx_pos, np.float64)
    edges, en = O._c(os_.edges, np.int32), O._c(os_.edge_n, np.float64)
    got = lib.orc_validate(i32(os_.T), p(g.tv), p(os_.tri_face), p(g.plane), i32(os_.F), i32(os_.E), i32(len(tx)),
                           i32(len(rx)), p(os_.face_off), p(os_.face_tris), p(g.verts), p(edges), p(en), p(tx), p(rx),
                           ctypes.c_double(250.0), i32(n), p(keys), p(valid), p(amb), p(tri), p(pts))
    assert got == nbad
    assert np.all(valid[1:] == 0) and np.all(amb[1:] == 0) and np.all(tri[1:] == -1)
    assert valid[0] in (0, 1)
    got = lib.orc_image_points(i32(n), p(keys), i32(os_.F), i32(os_.E), i32(len(tx)), i32(len(rx)), p(g.plane),
                               p(g.verts), p(edges), p(en), p(tx), p(rx), p(pts))
    assert got == nbad and np.all(pts[1:] == 0.0)
    a = np.zeros((n, 1, 2))
    tau, fd, aod, aoa = np.zeros(n), np.zeros((n, 1)), np.zeros((n, 2)), np.zeros((n, 2))
    zeros3 = np.zeros((max(1, len(tx)), 3))
    got = lib.orc_eval(i32(n), p(keys), i32(os_.F), i32(os_.E), i32(len(tx)), i32(len(rx)), p(pts), p(g.plane),
                       p(os_.face_material), p(os_.face_dyn), p(np.zeros((1, 3))), p(os_.materials),
                       p(os_.material_refl), p(g.verts), p(edges), p(en), p(tx), p(O._c(zeros3, np.float64)),
                       p(O._c(fr.tx_orient, np.float64)), p(rx), p(O._c(fr.rx_vel, np.float64)), i32(0), i32(1),
                       p(np.array([28e9])), p(a), p(tau), p(fd), p(aod), p(aoa))
    assert got == nbad
    assert np.all(np.isnan(tau[1:])) and np.isfinite(tau[0])
    for row in keys[1:]:
        with pytest.raises(O.MalformedKey) as e:
            O.validate(os_, g, row[None], fr.tx_pos, fr.rx_pos)
        assert str(row.tolist()) in str(e.value)


@pytest.mark.skipif(bool(os.environ.get("EMRT_ORACLE_LIB")), reason="already inside the sanitized run")
def test_pin_suites_under_address_and_ub_sanitizers(tmp_path):
    lib = O.build(sanitize=True, out=str(tmp_path / "liborc_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    env = dict(os.environ)
    env["EMRT_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = " ".join(x for x in (asan, env.get("LD_PRELOAD", "")) if x)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    # -s: a sanitizer report ends the process, so it must not sit in pytest's capture
    cmd = [sys.executable, "-m", "pytest", "-s", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *PIN_FILES, "tests/test_oracle_sanitized.py::test_malformed_keys_rejected_in_c"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-3000:]).strip()
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
