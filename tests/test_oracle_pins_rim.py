"""Pins of the oracle's rim-circle contact (the cylindrical wheels of Sec. IV-D's
terrain robot): each wheel touches with the two circles of its rims, and a
circle of radius r and axis a reaches r sqrt(1 - (n . a)^2) below its centre
along a contact normal n.

None of these checks uses that formula.  The gap is read back from the
oracle's residual (the normal row of a penetrating contact at lambda = 0) and
compared with a brute-force minimum over 20,000 points of the rim, at q- and
after a rotation of the iterate; the contact point's slip velocity, from the
friction rows, with the velocity of the brute-force lowest rim point; the
gap's Jacobian with central differences of the gap; a flat heightmap with the
plane; an upright wheel at rest with the weight it carries; the contact's
activation at q- with the brute-force lowest rim point; and the exact step
adjoint, whose q- and u- cotangents pass through the rim's depth and lever,
with central differences of the step on single rim contacts on the plane, on
the obstacle box's side face and over its top edge, and on a mesh edge and a
mesh vertex.  Five plausible
mistakes in the oracle's rim code, each planted in a copy of it, fail one of
these pins.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

R_WHEEL = 0.1


def _quat_axis_angle(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    s = math.sin(0.5 * ang)
    return np.array([axis[0] * s, axis[1] * s, axis[2] * s, math.cos(0.5 * ang)])


def _rot(q):
    x, y, z, w = np.asarray(q, float) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _qmul(a, b):
    ax, ay, az, aw = a
    bx, by, bz, bw = b
    return np.array([aw * bx + ax * bw + ay * bz - az * by, aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw, aw * bw - ax * bx - ay * by - az * bz])


def _pose_after(q, u, h):
    """Pose at the iterate u: x + h v, and the quaternion q + (h/2) w (x) q normalised
    (world-frame angular velocity w), the kinematic substitution of Eq. (1)."""
    x = q[:3] + h * u[:3]
    dq = 0.5 * h * _qmul(np.array([u[3], u[4], u[5], 0.0]), q[3:7])
    qn = q[3:7] + dq
    return x, qn / np.linalg.norm(qn)


def _rim_points(x, quat, local, axis_b, r, n_pts=20000):
    R = _rot(quat)
    e = np.asarray(axis_b, float)
    t = np.cross(e, [1.0, 0.0, 0.0])
    if np.linalg.norm(t) < 1e-6:
        t = np.cross(e, [0.0, 0.0, 1.0])
    u1 = t / np.linalg.norm(t)
    u2 = np.cross(e, u1)
    th = np.linspace(0.0, 2.0 * math.pi, n_pts, endpoint=False)
    pl = np.asarray(local, float)[None, :] + r * (np.cos(th)[:, None] * u1 + np.sin(th)[:, None] * u2)
    return x[None, :] + pl @ R.T


def _disc_world(q, mu=0.8, local=(0.0, 0.0, 0.0), kind=scenes.SLOT_PLANE, axis=(0.0, 1.0, 0.0), hm_index=-1,
                obstacle=None):
    """One free wheel body with a single rim-circle slot (against the plane, a
    heightmap, or the given static box (centre, half extents))."""
    wd = scenes.World(contact_cap=4)
    b = wd.add_body(1.0, scenes.cylinder_inertia_y(1.0, R_WHEEL, 0.05), tuple(q))
    if obstacle is not None:
        wd.add_obstacle(*obstacle)
    feature = 0 if kind in (scenes.SLOT_HEIGHTMAP, scenes.SLOT_BOX) else -1
    wd.add_slot(kind, b, local=local, radius=R_WHEEL, mu=mu, axis=axis, feature=feature)
    wd.knots = np.zeros((0, scenes.ROBOT_KNOTS))
    wd.heightmap = hm_index
    return wd


def _gap_from_residual(F, nu, eps):
    """Gap g of the first contact's normal row at lambda = 0: the row is
    g - sqrt(g^2 + eps^2), which inverts to g = (r^2 - eps^2) / (2 r)."""
    r = F[nu]
    assert r < -1e-6, "the pin needs a penetrating contact (a well-conditioned inversion)"
    return (r * r - eps * eps) / (2.0 * r)


def _inspect_gap(batch, P, u_it):
    res = oracle.inspect(batch, P, 0, batch.q0, batch.u0, None, u_it=u_it, lam_it=np.zeros(3))
    assert res["m"] == 3
    return _gap_from_residual(res["F"], res["nu"], P["eps"]), res


@pytest.mark.parametrize("tilt", [0.0, 0.3, 1.0])
def test_rim_gap_on_the_plane_is_the_lowest_rim_point(tilt):
    """A rim circle tilted by `tilt` about x (its axis (0, cos, sin)) just below
    the plane: the gap at q- and at an iterate that spins it about its axle and
    tips it further equals the lowest of 20,000 rim points."""
    P = scenes.solver_params()
    q0 = np.r_[[0.2, -0.1, R_WHEEL * math.cos(tilt) - 0.004], _quat_axis_angle((1, 0, 0), tilt)]
    b = scenes.pack([_disc_world(q0)])
    for u in (np.zeros(6), np.array([0.3, -0.2, -0.05, 0.0, 4.0, 0.0]),
              np.array([0.1, 0.0, -0.02, 0.7, 2.0, -0.4])):
        g, _ = _inspect_gap(b, P, u)
        x, qq = _pose_after(q0, u, P["h"])
        pts = _rim_points(x, qq, (0, 0, 0), (0, 1, 0), R_WHEEL)
        assert abs(g - pts[:, 2].min()) < 1e-8, (tilt, u, g, pts[:, 2].min())


def test_rim_gap_on_the_obstacle_top_face():
    """A tilted rim circle over the static box's top face (its centre above the
    face's interior): the gap equals the least height of the rim's points above
    the face, at q- and at a rotated iterate."""
    P = scenes.solver_params()
    top = 0.15
    box = ((0.0, 0.0, 0.5 * top), (0.6, 0.4, 0.5 * top))
    tilt = 0.4
    q0 = np.r_[[0.1, -0.05, top + R_WHEEL * math.cos(tilt) - 0.003], _quat_axis_angle((1, 0.3, 0), tilt)]
    b = scenes.pack([_disc_world(q0, kind=scenes.SLOT_BOX, obstacle=box)])
    for u in (np.zeros(6), np.array([0.2, -0.1, -0.03, 0.4, 3.0, -0.2])):
        g, _ = _inspect_gap(b, P, u)
        x, qq = _pose_after(q0, u, P["h"])
        pts = _rim_points(x, qq, (0, 0, 0), (0, 1, 0), R_WHEEL)
        assert abs(g - (pts[:, 2].min() - top)) < 1e-8


def test_rim_facing_the_plane_touches_with_its_centre_height():
    """A rim circle lying flat (axis vertical): every rim point is at the
    centre's height, and so is the gap."""
    P = scenes.solver_params()
    q0 = np.r_[[0.0, 0.0, -0.003], _quat_axis_angle((1, 0, 0), 0.5 * math.pi)]
    b = scenes.pack([_disc_world(q0)])
    g, _ = _inspect_gap(b, P, np.zeros(6))
    assert abs(g - (-0.003)) < 1e-12


def test_rim_gap_on_a_sideways_mesh_slope():
    """A heightmap sloping across the wheel's axle (heights s y): the face
    under the rim has normal (0, -s, 1)/sqrt(1 + s^2), and the gap equals the
    least signed distance of the rim's points from that face."""
    s = 0.4
    n = 40
    sp = 0.05
    origin = (-1.0, -1.0)
    ys = origin[1] + sp * np.arange(n)
    hm = scenes.Heightmap(n=n, spacing=sp, origin=origin, heights=np.tile(s * ys, (n, 1)))
    P = scenes.solver_params()
    x0 = np.array([0.013, 0.021, 0.0])
    nrm = np.array([0.0, -s, 1.0]) / math.sqrt(1 + s * s)
    # place the rim 3 mm into the face: centre height from the brute-force depth
    q_rot = _quat_axis_angle((0, 0, 1), 0.2)
    pts = _rim_points(np.zeros(3), q_rot, (0, 0, 0), (0, 1, 0), R_WHEEL)
    depth = -(pts @ nrm).min()
    x0[2] = s * x0[1] + (depth - 0.003) / nrm[2]
    q0 = np.r_[x0, q_rot]
    b = scenes.pack([_disc_world(q0, kind=scenes.SLOT_HEIGHTMAP, hm_index=0)], [hm])
    for u in (np.zeros(6), np.array([0.2, 0.1, -0.03, 0.2, 3.0, 0.5])):
        g, _ = _inspect_gap(b, P, u)
        x, qq = _pose_after(q0, u, P["h"])
        pts = _rim_points(x, qq, (0, 0, 0), (0, 1, 0), R_WHEEL)
        a0 = np.array([origin[0], origin[1], s * origin[1]])
        assert abs(g - ((pts - a0) @ nrm).min()) < 1e-8


def test_rim_gap_jacobian_and_slip_velocity():
    """The normal row's Jacobian is (1/h) of the gap's derivative in u (central
    differences of the gap read back from the residual), and the friction rows
    give the tangential velocity of the lowest rim point at the iterate."""
    P = scenes.solver_params()
    h = P["h"]
    tilt = 0.25
    q0 = np.r_[[0.0, 0.0, R_WHEEL * math.cos(tilt) - 0.005], _quat_axis_angle((1, 0.2, 0), tilt)]
    b = scenes.pack([_disc_world(q0)])
    u = np.array([0.4, -0.3, -0.02, 0.5, 3.0, -0.7])
    g, res = _inspect_gap(b, P, u)
    J = res["J"]
    fd = np.zeros(6)
    d = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = d
        fd[k] = (_inspect_gap(b, P, u + e)[0] - _inspect_gap(b, P, u - e)[0]) / (2 * d)
    np.testing.assert_allclose(J[0] * h, fd, rtol=0, atol=1e-7)
    # slip velocity of the contact point: the lowest rim point, moving with the body
    x, qq = _pose_after(q0, u, h)
    pts = _rim_points(x, qq, (0, 0, 0), (0, 1, 0), R_WHEEL, n_pts=200000)
    pc = pts[np.argmin(pts[:, 2])]
    vc = u[:3] + np.cross(u[3:], pc - x)
    vt = vc - vc[2] * np.array([0.0, 0.0, 1.0])
    slip = np.array([J[1] @ u, J[2] @ u])
    assert abs(np.linalg.norm(slip) - np.linalg.norm(vt)) < 2e-5 * max(1.0, np.linalg.norm(vt))


@pytest.mark.parametrize("wheels", ["sphere", "cylinder"])
def test_flat_terrain_with_rim_circles_reproduces_the_plane(wheels):
    """The robot with sphere or cylindrical wheels on a flat heightmap moves
    exactly as on the plane z = 0 with the same proxies."""
    hm = scenes.Heightmap(n=40, spacing=0.05, origin=(-1.0, -1.0), heights=np.zeros((40, 40)))
    rng = np.random.default_rng(1)
    knots = rng.uniform(-2, 2, size=(4, scenes.ROBOT_KNOTS))
    tw = scenes.robot_terrain_world(None, hm, 0, yaw=0.2, knots=knots, start=(0.1, 0.05), wheels=wheels)
    pw = scenes.robot_world(None, yaw=0.2, knots=knots, with_obstacle=False, wheels=wheels)
    pw.q0 = [list(q) for q in tw.q0]
    bt, bp = scenes.pack([tw], [hm]), scenes.pack([pw])
    P = scenes.solver_params(k_max=64)
    B = oracle.spline_basis(12, scenes.ROBOT_KNOTS, P["h"])
    qt, ut, lt = bt.q0.copy(), bt.u0.copy(), np.zeros(bt.n_lam)
    qp, up, lp = bp.q0.copy(), bp.u0.copy(), np.zeros(bp.n_lam)
    for k in range(6):
        c = knots.reshape(-1, scenes.ROBOT_KNOTS) @ B[k]
        ot = oracle.step_forward(bt, P, qt, ut, lt, c)
        op = oracle.step_forward(bp, P, qp, up, lp, c)
        assert np.array_equal(ot["status"], op["status"])
        np.testing.assert_allclose(ot["u"], op["u"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(ot["q"], op["q"], rtol=0, atol=1e-12)
        qt, ut, lt = ot["q"], ot["u"], ot["lam"]
        qp, up, lp = op["q"], op["u"], op["lam"]


def test_upright_cylinder_rests_on_both_rims():
    """A free upright wheel (two rim circles 5 cm apart) on the plane settles
    at rest, each rim carrying half its weight: lambda_n = m g / 2 (the
    multipliers are forces: r_dyn = M~ (u - u-) - h (f_ext + J^T lambda))."""
    wd = scenes.World(contact_cap=4)
    m = 1.0
    b = wd.add_body(m, scenes.cylinder_inertia_y(m, R_WHEEL, 0.05), (0.0, 0.0, R_WHEEL, 0.0, 0.0, 0.0, 1.0))
    for o in (-0.025, 0.025):
        wd.add_slot(scenes.SLOT_PLANE, b, local=(0.0, o, 0.0), radius=R_WHEEL, mu=0.8, axis=(0.0, 1.0, 0.0))
    wd.knots = np.zeros((0, scenes.ROBOT_KNOTS))
    batch = scenes.pack([wd])
    P = scenes.solver_params(k_max=64, tol=1e-12)
    q, u, lam = batch.q0.copy(), batch.u0.copy(), np.zeros(batch.n_lam)
    for _ in range(5):
        o = oracle.step_forward(batch, P, q, u, lam, None)
        q, u, lam = o["q"], o["u"], o["lam"]
    assert o["n_act"][0] == 2
    np.testing.assert_allclose(u, 0.0, atol=1e-9)
    ln = lam[0::3][:2]
    np.testing.assert_allclose(ln, 0.5 * m * 9.81, rtol=1e-6)


def test_rim_circle_on_a_body_face_is_rejected():
    wd = scenes.World(contact_cap=4)
    a = wd.add_body(1.0, (1, 1, 1), (0, 0, 1, 0, 0, 0, 1))
    with pytest.raises(ValueError):
        wd.add_slot(scenes.SLOT_BODYFACE, a, radius=0.1, b=0, face_h=0.1, axis=(0, 1, 0))


@pytest.mark.parametrize("above,active", [(0.002, False), (-0.002, True)])
def test_rim_activation_uses_the_lowest_rim_point(above, active):
    """A contact is activated at q- when its gap (at rest) is within delta0: a
    rim circle tilted by 1 rad whose lowest point (brute force) is 2 mm above
    or below delta0 is inactive or active.  A sphere of the same radius would
    reach 4.6 cm lower and be active in both cases."""
    P = scenes.solver_params()
    q = np.r_[[0.1, 0.2, 0.0], _quat_axis_angle((1, 0, 0), 1.0)]
    low = _rim_points(np.zeros(3), q[3:], (0, 0, 0), (0, 1, 0), R_WHEEL)[:, 2].min()
    q[2] = P["delta0"] + above - low
    b = scenes.pack([_disc_world(q)])
    res = oracle.inspect(b, P, 0, b.q0, b.u0, None)
    assert (res["m"] == 3) == active, (above, res["m"])


# Plausible mistakes in the oracle's rim-circle code, each planted in a copy of
# the oracle, must fail at least one of the pins above.
def _pins_on_the_plane():
    for tilt in (0.3, 1.0):
        test_rim_gap_on_the_plane_is_the_lowest_rim_point(tilt)


def _pin_slip():
    test_rim_gap_jacobian_and_slip_velocity()


def _pin_activation():
    test_rim_activation_uses_the_lowest_rim_point(0.002, False)


RIM_PLANTS = [
    ("depth_without_sqrt", "  S sn = sqrt(s2);\n", "  S sn = s2;\n", [_pins_on_the_plane]),
    ("support_sign", "if (d) *d = (n - a * na) * (1.0 / sn);", "if (d) *d = (n + a * na) * (1.0 / sn);",
     [_pin_slip]),
    ("axis_not_rotated", "C.noff - rim_depth(C.n, qrot(qa, cst3<S>(C.ax.x, C.ax.y, C.ax.z)), C.r,",
     "C.noff - rim_depth(C.n, cst3<S>(C.ax.x, C.ax.y, C.ax.z), C.r,", [_pins_on_the_plane]),
    ("sphere_lever", "S(C.loc.z)}) - dsup * C.r;", "S(C.loc.z)}) - C.n * C.r;", [_pin_slip]),
    ("activation_gap_offset", "gap = gap + S.r - rim_depth(", "gap = gap - rim_depth(", [_pin_activation]),
]


@pytest.mark.parametrize("name,old,new,pins", RIM_PLANTS, ids=[p[0] for p in RIM_PLANTS])
def test_planted_rim_mistake_fails_its_pin(tmp_path, name, old, new, pins):
    from test_oracle_pins_geometry import planted
    with planted(tmp_path, old, new):
        for pin in pins:
            with pytest.raises(AssertionError):
                pin()
    for pin in pins:  # and the unplanted oracle passes them again
        pin()


def _step_adjoint_fd(b, P, q, u):
    """The oracle's exact step adjoint of a random linear loss of (q+, u+) against central
    differences of the converged step in every component of q- and u- (the active set
    unchanged by each perturbation).  Returns the relative deviation."""
    lam = np.zeros(b.n_lam)
    ref = oracle.step_forward(b, P, q, u, lam, None)
    assert ref["status"][0] & 1 and ref["n_act"][0] == 1, ref["status"]
    rng = np.random.default_rng(0)
    gq, gu = rng.normal(size=q.shape), rng.normal(size=u.shape)
    aq, au, _ = oracle.step_adjoint(b, P, q, u, lam, None, ref["u"], ref["lam"], gq, gu, mode=0)

    def loss(qq, uu):
        o = oracle.step_forward(b, P, qq, uu, lam, None)
        assert o["status"][0] & 1 and np.array_equal(o["act_slot"], ref["act_slot"])
        return float(np.sum(gq * o["q"]) + np.sum(gu * o["u"]))

    g = np.concatenate([aq.ravel(), au.ravel()])
    fd = np.zeros_like(g)
    for i in range(g.size):
        x = (q if i < q.size else u).copy()
        j = i if i < q.size else i - q.size
        d = 1e-6 * max(1.0, abs(x.flat[j]))
        xp, xm = x.copy(), x.copy()
        xp.flat[j] += d
        xm.flat[j] -= d
        lp = loss(xp, u) if i < q.size else loss(q, xp)
        lm = loss(xm, u) if i < q.size else loss(q, xm)
        fd[i] = (lp - lm) / (2 * d)
    return np.linalg.norm(fd - g) / np.linalg.norm(g)


def test_rim_step_adjoint_on_the_plane_matches_central_differences():
    """A rim circle tilted by 0.3 rad (n . a = sin 0.3, so the depth and the contact
    point turn with the axle), 2 mm into the plane, sliding and spinning under gravity
    (mu = 0.3, a sliding contact): the exact adjoint's q- and u- cotangents, which pass
    through the rim's depth and lever at q- and at the iterate, against central
    differences of the step."""
    P = scenes.solver_params(k_max=200, tol=1e-14)
    tilt = 0.3
    q0 = np.r_[[0.0, 0.0, R_WHEEL * math.cos(tilt) - 0.002], _quat_axis_angle((1, 0, 0), tilt)]
    b = scenes.pack([_disc_world(q0, mu=0.3)])
    u0 = np.array([[0.8, 0.3, -0.05, 0.4, 3.0, -0.5]])
    dev = _step_adjoint_fd(b, P, b.q0.copy(), u0)
    assert dev <= 1e-5, dev


def test_rim_step_adjoint_on_the_obstacle_side_face_matches_central_differences():
    """A rim circle yawed by 0.26 rad pressed 2 mm into the static box's -x face in zero
    gravity (n = -x, n . a = sin 0.26): the same check as on the plane, through the box
    feature's frame."""
    P = scenes.solver_params(k_max=200, tol=1e-14, gravity=(0.0, 0.0, 0.0))
    box = ((1.0, 0.0, 0.075), (0.6, 0.4, 0.075))
    yaw = 0.26
    x_face = box[0][0] - box[1][0]
    q0 = np.r_[[x_face - R_WHEEL * math.cos(yaw) + 0.002, 0.05, 0.075], _quat_axis_angle((0, 0, 1), yaw)]
    b = scenes.pack([_disc_world(q0, mu=0.3, kind=scenes.SLOT_BOX, obstacle=box)])
    u0 = np.array([[0.5, 0.2, 0.1, 0.3, 2.0, -0.4]])
    dev = _step_adjoint_fd(b, P, b.q0.copy(), u0)
    assert dev <= 1e-5, dev


def _rim_over_box_edge():
    """A rim circle (axis yawed by 0.26 rad) over the static box's -x top edge, its centre
    in the edge's region, 2 mm into the edge along n = (-1, 0, 1)/sqrt 2, the normal from
    the edge to the centre (it turns with the centre)."""
    box = ((1.0, 0.0, 0.075), (0.6, 0.4, 0.075))
    yaw = 0.26
    n = np.array([-1.0, 0.0, 1.0]) / math.sqrt(2.0)
    a = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
    depth = R_WHEEL * math.sqrt(1.0 - float(n @ a) ** 2)
    c = np.array([0.4, 0.05, 0.15]) + n * (depth - 0.002)
    q0 = np.r_[c, _quat_axis_angle((0, 0, 1), yaw)]
    return scenes.pack([_disc_world(q0, mu=0.3, kind=scenes.SLOT_BOX, obstacle=box)])


def test_rim_step_adjoint_over_the_obstacle_edge_matches_central_differences():
    """The rim circle over the box's edge, sliding along it under gravity: the normal, the
    depth and the lever all depend on q-; the exact adjoint against central differences."""
    P = scenes.solver_params(k_max=200, tol=1e-14)
    b = _rim_over_box_edge()
    u0 = np.array([[0.3, 0.6, -0.1, 0.2, 2.0, -0.3]])
    dev = _step_adjoint_fd(b, P, b.q0.copy(), u0)
    assert dev <= 1e-5, dev


def _rim_on_mesh_feature(kind):
    """A single rim circle (a wheel tipped by 0.4 rad about (1, 0.3, 0)) 2 mm into a convex
    mesh feature along a normal n from the feature to the centre: the edge of the ridge
    z = -|x| (n tipped 0.15 rad towards +x), or the vertex of the peak z = -(|x| + |y|)."""
    n_grid, sp = 9, 0.1
    xs = (np.arange(n_grid) - 4) * sp
    if kind == "ridge":
        heights = -np.abs(xs)[:, None] * np.ones(n_grid)[None, :]
        foot = np.array([0.0, 0.013, 0.0])
        n = np.array([math.sin(0.15), 0.0, math.cos(0.15)])
    else:
        heights = -(np.abs(xs)[:, None] + np.abs(xs)[None, :])
        foot = np.zeros(3)
        n = np.array([0.05, -0.04, 1.0]) / np.linalg.norm([0.05, -0.04, 1.0])
    hm = scenes.Heightmap(n=n_grid, spacing=sp, origin=(xs[0], xs[0]), heights=heights)
    quat = _quat_axis_angle((1, 0.3, 0), 0.4)
    a = _rot(quat) @ np.array([0.0, 1.0, 0.0])
    depth = R_WHEEL * math.sqrt(1.0 - float(n @ a) ** 2)
    q0 = np.r_[foot + n * (depth - 0.002), quat]
    return scenes.pack([_disc_world(q0, mu=0.3, kind=scenes.SLOT_HEIGHTMAP, hm_index=0)], [hm])


@pytest.mark.parametrize("kind", ["ridge", "peak"])
def test_rim_step_adjoint_on_mesh_edge_and_vertex_matches_central_differences(kind):
    """Rim circles on a mesh edge and a mesh vertex, whose normals turn with the wheel's
    centre: the exact adjoint against central differences of the step."""
    P = scenes.solver_params(k_max=200, tol=1e-14)
    b = _rim_on_mesh_feature(kind)
    u0 = np.array([[0.2, 0.4, -0.1, 0.3, 2.5, -0.2]])
    dev = _step_adjoint_fd(b, P, b.q0.copy(), u0)
    assert dev <= 1e-5, dev


def test_rim_parameter_cotangents_match_central_differences():
    """Eq. (17) with a model parameter as xi through a rim contact: the mass and the
    friction coefficient cotangents of a single rim circle sliding on the plane and
    over the obstacle box's top edge, against central differences of the step."""
    from test_oracle_pins import _param_fd
    P = scenes.solver_params(k_max=200, tol=1e-14)
    tilt = 0.3
    q0 = np.r_[[0.0, 0.0, R_WHEEL * math.cos(tilt) - 0.002], _quat_axis_angle((1, 0, 0), tilt)]
    plane = scenes.pack([_disc_world(q0, mu=0.3)])
    plane.u0 = np.array([[0.8, 0.3, -0.05, 0.4, 3.0, -0.5]])
    edge = _rim_over_box_edge()
    edge.u0 = np.array([[0.3, 0.6, -0.1, 0.2, 2.0, -0.3]])
    for b in (plane, edge):
        assert _param_fd(b, P, None) == 2  # the mass and the slot's friction coefficient
