"""Pins of the CPU oracle's remaining residual terms against closed forms (no GPU).

* The explicit gyroscopic term of f_ext (Sec. III-A, Eq. (2)): a torque-free
  body spinning off its principal axes.
* Contact with the static obstacle box (Sec. III-B, Eq. (4) on a non-plane
  feature): a sphere on the top face, against a side face, over an edge, over
  a vertex, and a point inside the box.
* Box-on-box contact (Sec. III-B, Eqs. (4) and (7) with the face of a moving
  body): a resting stack and a box sliding on a box.

Each closed form is written here with numpy from the backward-Euler step of
Eqs. (1)-(2) and the complementarity conditions, not from the oracle's code.
The planted-mistake tests compile a copy of the oracle with one term changed
(the gyroscopic sign, the feature choice of the obstacle box, the inside normal,
the lower body's contact point) and check that the pin of that term fails.
"""
import contextlib
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import scenes
from test_oracle_pins import contact_lams, quat_R

G = 9.81
OBS_C, OBS_H = np.array([0.0, 0.0, 0.5]), np.array([0.5, 0.4, 0.5])  # obstacle centre, half extents


def _step(b, P, steps=1):
    q, u, lam = b.q0.copy(), b.u0.copy(), np.zeros(b.n_lam)
    outs = []
    for _ in range(steps):
        o = oracle.step_forward(b, P, q, u, lam, None)
        outs.append(o)
        q, u, lam = o["q"], o["u"], o["lam"]
    return outs


# ------------------------------------------------------------ gyroscopic term

def _spinning_body():
    wd = scenes.World(contact_cap=0)
    q = np.array([0.3, -0.2, 0.5, 0.8])
    q /= np.linalg.norm(q)
    wd.add_body(2.0, (0.1, 0.2, 0.3), (0.0, 0.0, 1.0, *q), (0.2, -0.1, 0.3, 1.3, -0.7, 2.1))
    return scenes.pack([wd])


def pin_gyroscopic():
    """Torque-free rigid body in zero gravity, spinning off its principal axes.
    With f_ext = -w- x (I_w w-) explicit at q- and M~ at q-, each step gives
    w+ = w- - h I_w^-1 (w- x I_w w-), then q+ = normalise(q- + h/2 (w+, 0) (x) q-)."""
    b = _spinning_body()
    P = scenes.solver_params(tol=1e-13, k_max=64, gravity=(0.0, 0.0, 0.0))
    h = P["h"]
    outs = _step(b, P, 4)
    x, q = np.array(b.q0[0, :3]), np.array(b.q0[0, 3:])
    v, w = np.array(b.u0[0, :3]), np.array(b.u0[0, 3:])
    I = np.diag(b.body_inertia[0])
    for o in outs:
        R = quat_R(q)
        Iw = R @ I @ R.T
        w = w - h * np.linalg.solve(Iw, np.cross(w, Iw @ w))
        x = x + h * v
        dq = np.concatenate([q[3] * w + np.cross(w, q[:3]), [-np.dot(w, q[:3])]])
        q = q + 0.5 * h * dq
        q /= np.linalg.norm(q)
        assert o["status"][0] & 1
        np.testing.assert_allclose(o["u"][0, 3:], w, rtol=0, atol=1e-11)
        np.testing.assert_allclose(o["u"][0, :3], v, rtol=0, atol=1e-12)
        np.testing.assert_allclose(o["q"][0, :3], x, rtol=0, atol=1e-12)
        np.testing.assert_allclose(o["q"][0, 3:], q, rtol=0, atol=1e-11)
    # the term is not negligible here: the spin changes by more than 1e-2 per step
    assert np.linalg.norm(outs[0]["u"][0, 3:] - b.u0[0, 3:]) > 1e-2


def test_gyroscopic_term_closed_form():
    pin_gyroscopic()


# ------------------------------------------------------ static obstacle box

def _sphere_vs_obstacle(p, v, r, mu=0.5):
    wd = scenes.World(contact_cap=1)
    bi = wd.add_body(1.0, (0.004, 0.004, 0.004), (*p, 0.0, 0.0, 0.0, 1.0), (*v, 0.0, 0.0, 0.0))
    o = wd.add_obstacle(tuple(OBS_C), tuple(OBS_H))
    wd.add_slot(scenes.SLOT_BOX, bi, radius=r, mu=mu, feature=o)
    return scenes.pack([wd])


def _closest_on_box(p):
    return np.clip(p, OBS_C - OBS_H, OBS_C + OBS_H)


def _approach_case(p, n, gap, speed=1.0, r=0.1):
    """A sphere of radius r whose centre is gap + r from the feature along n,
    moving at `speed` straight at it in zero gravity: the step closes the gap
    exactly, v+ = -(gap / h) n, with the normal impulse m (v+ - v-) . n / h and no
    friction (no slip, no torque: the force acts through the centre)."""
    b = _sphere_vs_obstacle(p, -speed * n, r)
    P = scenes.solver_params(tol=1e-13, k_max=64, gravity=(0.0, 0.0, 0.0))
    h = P["h"]
    o = _step(b, P)[0]
    assert o["status"][0] & 1 and o["n_act"][0] == 1
    want = -(gap / h) * n
    np.testing.assert_allclose(o["u"][0, :3], want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(o["u"][0, 3:], 0.0, atol=1e-9)
    lam = contact_lams(b, 0, o["lam"])[0]
    assert abs(lam[0] - (speed - gap / h) / h) < 1e-7, lam
    assert np.linalg.norm(lam[1:]) < 1e-7, lam


def pin_obstacle_top_face():
    """A sphere resting on the top face under gravity stays at rest with
    lambda_n = m g (the face is the plane z = top, normal +z)."""
    r = 0.1
    b = _sphere_vs_obstacle((0.1, 0.05, 1.0 + r), (0.0, 0.0, 0.0), r)
    P = scenes.solver_params(tol=1e-13, k_max=64)
    for o in _step(b, P, 3):
        assert o["status"][0] & 1
        np.testing.assert_allclose(o["u"][0], 0.0, atol=1e-9)
        lam = contact_lams(b, 0, o["lam"])[0]
        assert abs(lam[0] - G) < 1e-7 and np.linalg.norm(lam[1:]) < 1e-7, lam


def pin_obstacle_side_face():
    r, gap = 0.1, 0.02
    _approach_case((0.5 + r + gap, 0.1, 0.5), np.array([1.0, 0.0, 0.0]), gap)


def pin_obstacle_edge():
    """Beyond the +x face and above the top: the closest feature is the edge
    x = 0.5, z = 1, and the normal is (P - closest point) / |P - closest point|."""
    r, gap, th = 0.1, 0.02, math.radians(35.0)
    n = np.array([math.cos(th), 0.0, math.sin(th)])
    p = np.array([0.5, 0.1, 1.0]) + (r + gap) * n
    assert np.allclose(_closest_on_box(p), [0.5, 0.1, 1.0])
    _approach_case(p, n, gap)


def pin_obstacle_vertex():
    r, gap = 0.1, 0.03
    n = np.array([1.0, 0.7, 1.2])
    n /= np.linalg.norm(n)
    corner = OBS_C + OBS_H
    p = corner + (r + gap) * n
    assert np.allclose(_closest_on_box(p), corner)
    _approach_case(p, n, gap)


def pin_obstacle_inside():
    """A point 0.03 m inside the box, nearest to its +x face, at rest in zero
    gravity: the step pushes it out along +x to the face, v+ = (0.03 / h) e_x."""
    b = _sphere_vs_obstacle((0.47, 0.0, 0.5), (0.0, 0.0, 0.0), 0.0)
    P = scenes.solver_params(tol=1e-13, k_max=64, gravity=(0.0, 0.0, 0.0))
    h = P["h"]
    o = _step(b, P)[0]
    assert o["status"][0] & 1
    np.testing.assert_allclose(o["u"][0, :3], [0.03 / h, 0.0, 0.0], rtol=0, atol=1e-9)
    lam = contact_lams(b, 0, o["lam"])[0]
    assert abs(lam[0] - 0.03 / h / h) < 1e-7 and np.linalg.norm(lam[1:]) < 1e-7, lam


OBSTACLE_PINS = {"top": pin_obstacle_top_face, "side": pin_obstacle_side_face, "edge": pin_obstacle_edge,
                 "vertex": pin_obstacle_vertex, "inside": pin_obstacle_inside}


@pytest.mark.parametrize("case", sorted(OBSTACLE_PINS))
def test_obstacle_contact_closed_form(case):
    OBSTACLE_PINS[case]()


# ------------------------------------------------------------- box on box

def _resting_stack(n, seed=4):
    wd = scenes.stack_world(np.random.default_rng(seed), n)
    wd.u0 = [(0.0,) * 6 for _ in wd.u0]
    return scenes.pack([wd])


def pin_resting_stack():
    """A stack of boxes at rest stays at rest (u+ = 0), and the normal forces
    under each box sum to the weight of that box and all boxes above it; no
    friction acts.  The split over a box's four corners is not unique, the
    per-layer sums are."""
    n = 5
    b = _resting_stack(n)
    P = scenes.solver_params(tol=1e-11, k_max=64)  # the residual of a five-box stack floors near 5e-13
    masses = b.body_mass
    for o in _step(b, P, 2):
        assert o["status"][0] & 1
        np.testing.assert_allclose(o["u"], 0.0, atol=1e-9)
        lam = contact_lams(b, 0, o["lam"])
        for i in range(n):
            layer = lam[4 * i:4 * i + 4]
            assert abs(layer[:, 0].sum() - G * masses[i:].sum()) < 1e-7 * G * masses.sum(), (i, layer)
            assert np.linalg.norm(layer[:, 1:].sum(0)) < 1e-7, (i, layer)


def _sliding_pair(v0, mu):
    """A 0.2 m cube (1 kg) on the middle of a 0.5 m cube (5 kg) on the ground,
    both with friction coefficient mu, the top cube moving at v0 along x."""
    wd = scenes.World(contact_cap=8)
    eb, et, mb, mt = 0.5, 0.2, 5.0, 1.0
    lo = wd.add_body(mb, scenes.box_inertia(mb, eb, eb, eb), (0.0, 0.0, 0.5 * eb, 0.0, 0.0, 0.0, 1.0))
    up = wd.add_body(mt, scenes.box_inertia(mt, et, et, et), (0.0, 0.0, eb + 0.5 * et, 0.0, 0.0, 0.0, 1.0),
                     (v0, 0.0, 0.0, 0.0, 0.0, 0.0))
    for sx in (-1, 1):
        for sy in (-1, 1):
            wd.add_slot(scenes.SLOT_PLANE, lo, local=(sx * 0.5 * eb, sy * 0.5 * eb, -0.5 * eb), mu=mu)
    for sx in (-1, 1):
        for sy in (-1, 1):
            wd.add_slot(scenes.SLOT_BODYFACE, up, local=(sx * 0.5 * et, sy * 0.5 * et, -0.5 * et), mu=mu, b=lo,
                        face_h=0.5 * eb)
    return scenes.pack([wd]), mb, mt


def pin_box_sliding_on_box():
    """The top cube loses mu g h of speed per step until it sticks; the bottom
    cube is held by static friction with the ground (mu (m_t + m_b) g exceeds the
    mu m_t g the top cube drags it with) and stays at rest.  Normal forces: m_t g
    under the top cube, (m_t + m_b) g under the bottom one."""
    v0, mu = 0.7, 0.3
    b, mb, mt = _sliding_pair(v0, mu)
    P = scenes.solver_params(tol=1e-11, k_max=64)
    h = P["h"]
    speed = v0
    for k, o in enumerate(_step(b, P, 4)):
        speed = max(speed - mu * G * h, 0.0)
        assert o["status"][0] & 1, k
        np.testing.assert_allclose(o["u"][1, :3], [speed, 0.0, 0.0], rtol=0, atol=1e-9)
        np.testing.assert_allclose(o["u"][1, 3:], 0.0, atol=1e-9)
        np.testing.assert_allclose(o["u"][0], 0.0, atol=1e-9)
        lam = contact_lams(b, 0, o["lam"])
        assert abs(lam[4:, 0].sum() - mt * G) < 1e-7, (k, lam)
        assert abs(lam[:4, 0].sum() - (mt + mb) * G) < 1e-7, (k, lam)
        if speed > 0:  # sliding: the friction force on the top cube is mu m_t g
            assert abs(np.linalg.norm(lam[4:, 1:].sum(0)) - mu * mt * G) < 1e-7, (k, lam)


def test_resting_stack_closed_form():
    pin_resting_stack()


def test_box_sliding_on_box_closed_form():
    pin_box_sliding_on_box()


# ----------------------------------------------------------- planted mistakes

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ostrich_ref.cpp")


@contextlib.contextmanager
def planted(tmp_path, old, new):
    """The oracle with one source snippet replaced, swapped in for the duration."""
    src = open(_SRC).read()
    assert src.count(old) == 1, old
    cpp = tmp_path / "planted.cpp"
    so = tmp_path / "libplanted.so"
    cpp.write_text(src.replace(old, new))
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", os.path.dirname(_SRC), "-o",
                           str(so), str(cpp)])
    L = ctypes.CDLL(str(so))
    for name in ("ostrich_ref_step_forward", "ostrich_ref_step_adjoint", "ostrich_ref_step_adjoint_params",
                 "ostrich_ref_spline_basis", "ostrich_ref_rollout", "ostrich_ref_rollout_shaped",
                 "ostrich_ref_inspect"):
        getattr(L, name).restype = ctypes.c_int32
    saved = oracle.lib()
    oracle._lib = L
    try:
        yield
    finally:
        oracle._lib = saved


PLANTS = [
    ("gyro_sign", "V3<T> gyro = -cross(wm,", "V3<T> gyro = cross(wm,", [pin_gyroscopic]),
    ("box_feature", "F.flags[i] = pv < lo ? -1 : (pv > hi ? 1 : 0);", "F.flags[i] = pv < lo ? -1 : 0;",
     [pin_obstacle_edge, pin_obstacle_vertex]),
    ("inside_normal", "      e[i] = F.in_side;", "      e[i] = -F.in_side;", [pin_obstacle_inside]),
    ("face_point", "if (C.kind == 2) return dot(C.n, P - (xb + qrot(qb, C.lb))) - C.r;",
     "if (C.kind == 2) return dot(C.n, P - (xb - qrot(qb, C.lb))) - C.r;",
     [pin_resting_stack, pin_box_sliding_on_box]),
]


@pytest.mark.parametrize("name,old,new,pins", PLANTS, ids=[p[0] for p in PLANTS])
def test_planted_mistake_fails_its_pin(tmp_path, name, old, new, pins):
    with planted(tmp_path, old, new):
        for pin in pins:
            with pytest.raises(AssertionError):
                pin()
    for pin in pins:  # and the unplanted oracle passes them again
        pin()
