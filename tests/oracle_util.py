"""Helpers shared by the oracle pins (test infrastructure)."""
import numpy as np

from synth.city import Frame

C0 = 299792458.0


def static_frame(tx, rx, rx_vel=None, tx_vel=None, obj_xform=None, obj_vel=None, tx_orient=None):
    tx = np.asarray(tx, np.float64).reshape(-1, 3)
    rx = np.asarray(rx, np.float64).reshape(-1, 3)
    return Frame(
        t=0.0,
        obj_xform=np.zeros((0, 3, 4)) if obj_xform is None else np.asarray(obj_xform, np.float64),
        obj_vel=np.zeros((0, 3)) if obj_vel is None else np.asarray(obj_vel, np.float64),
        tx_pos=tx,
        tx_vel=np.zeros_like(tx) if tx_vel is None else np.asarray(tx_vel, np.float64).reshape(-1, 3),
        rx_pos=rx,
        rx_vel=np.zeros_like(rx) if rx_vel is None else np.asarray(rx_vel, np.float64).reshape(-1, 3),
        tx_orient=np.zeros((len(tx), 2)) if tx_orient is None else np.asarray(tx_orient, np.float64),
    )


def spec_key(tx, rx, faces):
    faces = list(faces)
    return [tx, rx, 1 if faces else 0, len(faces)] + faces + [-1] * (5 - len(faces))


def key_set(keys):
    return {tuple(int(x) for x in k) for k in np.asarray(keys).reshape(-1, 9)}
