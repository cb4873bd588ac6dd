"""Hand-worked single steps of the oracle's walk (the step rules of the Monte Carlo
method: free flight through transparent pores and attenuating solid, the first
nearest face in the order x, y, z, an interaction when the sampled free path is at
most the distance to the face, periodic lateral faces and axial escape).

Each case starts the oracle from a hand-made state on a hand-made mask and checks the
event, the voxel, the offsets and the remaining optical depth against values worked
out by hand, so a swapped axis, a wrong tie rule, a dropped clamp or a wrong sign
fails one of them.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle

W1 = 2 ** 31
EV = {v: k for k, v in oracle.EVENTS.items()}


def state(ix, iy, iz, f, u, tau, w=W1):
    s = np.zeros((), dtype=oracle.STATE_DTYPE)
    s["ix"], s["iy"], s["iz"] = ix, iy, iz
    s["fx"], s["fy"], s["fz"] = f
    s["ux"], s["uy"], s["uz"] = u
    s["tau"], s["w"] = tau, w
    return s


def step(mask, st, mu_s=0.5, mu_a=0.25, g=0.0):
    ev, new, _ = oracle.step_from(mask, mu_s, mu_a, g, 0, st, seed=1)
    return oracle.EVENTS[ev], new


def test_pore_flight_along_x_and_lateral_wrap():
    m = np.ones((2, 2, 2), dtype=np.uint8)                     # all pore: no optical depth is used
    ev, s = step(m, state(0, 0, 0, (0.25, 0.5, 0.0), (1.0, 0.0, 0.0), tau=3.0))
    assert ev == "face_x" and (s["ix"], s["iy"], s["iz"]) == (1, 0, 0)
    assert s["fx"] == 0.0 and s["fy"] == 0.5 and s["fz"] == 0.0
    assert s["tau"] == 3.0 and s["l_void"] == 0.75 and s["l_solid"] == 0.0
    ev, s = step(m, s)                                         # a full voxel, then the periodic face
    assert ev == "face_x" and s["ix"] == 0 and s["fx"] == 0.0 and s["l_void"] == 1.75
    back = state(0, 1, 1, (0.5, 0.25, 0.5), (0.0, -1.0, 0.0), tau=3.0)
    ev, s = step(m, back)
    assert ev == "face_y" and s["iy"] == 0 and s["fy"] == 1.0   # entering from the far face
    ev, s = step(m, s)
    assert ev == "face_y" and s["iy"] == 1 and s["fy"] == 1.0   # wrapped to the last row


def test_equal_face_distances_take_x_then_y_then_z():
    m = np.ones((2, 2, 2), dtype=np.uint8)
    u = 1.0 / math.sqrt(3.0)
    ev, s = step(m, state(0, 0, 0, (0.5, 0.5, 0.5), (u, u, u), tau=3.0))
    assert ev == "face_x" and (s["ix"], s["iy"], s["iz"]) == (1, 0, 0)
    # the other two axes reach their faces within rounding: they follow at once, y before z
    ev, s = step(m, s)
    assert ev == "face_y" and s["iy"] == 1 and abs(s["l_void"] - 0.5 * math.sqrt(3.0)) < 1e-12
    ev, s = step(m, s)
    assert ev == "face_z" and s["iz"] == 1
    assert abs(s["l_void"] - 0.5 * math.sqrt(3.0)) < 1e-12


def test_solid_voxel_uses_optical_depth():
    m = np.ones((3, 1, 1), dtype=np.uint8)
    m[1] = 0                                                   # pore, solid, pore along z
    mu_t = 0.5 + 0.25
    ev, s = step(m, state(0, 0, 0, (0.5, 0.5, 0.0), (0.0, 0.0, 1.0), tau=2.0))
    assert ev == "face_z" and s["iz"] == 1 and s["tau"] == 2.0 and s["l_void"] == 1.0
    ev, s = step(m, s)                                         # the whole solid voxel: tau falls by mu_t
    assert ev == "face_z" and s["iz"] == 2 and s["tau"] == 2.0 - mu_t and s["l_solid"] == 1.0
    ev, s = step(m, s)                                         # the last pore voxel, then out
    assert ev == "esc_T" and s["tau"] == 2.0 - mu_t and s["l_void"] == 2.0


def test_interaction_inside_the_voxel_and_implicit_capture():
    m = np.zeros((1, 1, 1), dtype=np.uint8)                    # one solid voxel
    # free path tau / mu_t = 0.3 / 0.75 = 0.4 < 0.9 to the face: an interaction at fz = 0.5
    ev, s = step(m, state(0, 0, 0, (0.5, 0.5, 0.1), (0.0, 0.0, 1.0), tau=0.3))
    assert ev == "scatter" and s["iz"] == 0 and abs(s["fz"] - 0.5) < 1e-15 and s["k"] == 1
    # survival mu_s / mu_t = 2/3 quantised to round(2^32 * 2/3) = 2863311531, then
    # floor((2^31 * 2863311531 + 2^31) / 2^32) = 1431655766
    assert s["w"] == 1431655766
    assert abs(s["ux"] ** 2 + s["uy"] ** 2 + s["uz"] ** 2 - 1.0) < 1e-12


def test_free_path_equal_to_the_face_distance_is_an_interaction():
    m = np.zeros((1, 1, 1), dtype=np.uint8)
    # mu_t = 0.5 (no absorption): tau 0.25 reaches exactly the face 0.5 away
    ev, s = step(m, state(0, 0, 0, (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), tau=0.25), mu_s=0.5, mu_a=0.0)
    assert ev == "scatter" and s["iz"] == 0 and s["fz"] == 1.0 and s["w"] == W1


@pytest.mark.parametrize("iz,uz,event", [(0, -1.0, "esc_R"), (3, 1.0, "esc_T")])
def test_axial_faces_are_escapes(iz, uz, event):
    m = np.ones((4, 2, 2), dtype=np.uint8)
    ev, s = step(m, state(1, 1, iz, (0.5, 0.5, 0.5), (0.0, 0.0, uz), tau=1.0))
    assert ev == event and s["l_void"] == 0.5
