"""Seeded synthetic scenes for the batched backward-Euler contact step.

This module only *describes* worlds (bodies, joints, contact candidate slots,
static obstacles, initial states, controls and loss targets) and packs many
worlds into flat world-major arrays.  It holds none of the simulation
arithmetic: both the CPU oracle and the GPU library consume the same packed
bytes produced here.

Scene shapes follow the paper's workloads (a box sliding on a plane, a wheeled
robot driven over a pallet-height box obstacle, stacks of boxes); the paper's
own robot and dataset are not public, so these synthetic scenes stand in for
them.

Conventions (shared by every consumer of the packed arrays):
  * per-body configuration q = (x, y, z, qx, qy, qz, qw)  -- position and a
    unit quaternion in (x, y, z, w) order;
  * per-body velocity u = (vx, vy, vz, wx, wy, wz) -- linear velocity of the
    centre of mass and angular velocity, both in the world frame;
  * gravity is a batch parameter (default (0, 0, -9.81)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# contact slot kinds
SLOT_PLANE = 0      # proxy sphere/point of body a against the ground plane z = 0
SLOT_BOX = 1        # proxy of body a against a static axis-aligned box obstacle
SLOT_BODYFACE = 2   # proxy of body a against the local +z face of body b
SLOT_HEIGHTMAP = 3  # proxy of body a against a triangle-mesh heightmap

# actuator modes per joint
ACT_NONE = 0
ACT_TORQUE = 1
ACT_SERVO_VEL = 2
ACT_TORQUE_DAMPED = 3   # torque from the control plus a velocity servo row with target 0
ACT_SERVO_POS = 4       # position servo: the control is the target joint angle (gains k_p, k_d)

JOINT_FRAME_LEN = 18   # anchor_a, anchor_b, axis_b, perp1_a, perp2_a, axis_a
SLOT_INT_LEN = 4       # kind, body_a, body_b, feature index
SLOT_REAL_LEN = 9      # local offset (3), radius, mu, face half-height, rim-circle axis (3; zero: sphere)

GRAVITY = (0.0, 0.0, -9.81)


def box_inertia(m: float, sx: float, sy: float, sz: float):
    """Principal moments of a solid box with full edge lengths sx, sy, sz."""
    return (m * (sy * sy + sz * sz) / 12.0,
            m * (sx * sx + sz * sz) / 12.0,
            m * (sx * sx + sy * sy) / 12.0)


def cylinder_inertia_y(m: float, r: float, w: float):
    """Principal moments of a solid cylinder whose axis is the local y axis."""
    side = m * (3.0 * r * r + w * w) / 12.0
    return (side, 0.5 * m * r * r, side)


def yaw_quat(yaw: float):
    return (0.0, 0.0, math.sin(0.5 * yaw), math.cos(0.5 * yaw))


@dataclasses.dataclass
class World:
    """One world: rigid bodies, revolute joints, contact slots, obstacles."""
    mass: List[float] = dataclasses.field(default_factory=list)
    inertia: List[Sequence[float]] = dataclasses.field(default_factory=list)
    q0: List[Sequence[float]] = dataclasses.field(default_factory=list)
    u0: List[Sequence[float]] = dataclasses.field(default_factory=list)
    joints: List[dict] = dataclasses.field(default_factory=list)
    slots: List[dict] = dataclasses.field(default_factory=list)
    obstacles: List[Sequence[float]] = dataclasses.field(default_factory=list)
    contact_cap: int = 16
    heightmap: int = -1
    loss_body: int = 0
    target: Sequence[float] = (0.0, 0.0)
    knots: Optional[np.ndarray] = None     # [n_ctrl, K] spline knots

    def add_body(self, mass, inertia, q, u=(0, 0, 0, 0, 0, 0)) -> int:
        self.mass.append(float(mass))
        self.inertia.append(tuple(float(v) for v in inertia))
        self.q0.append(tuple(float(v) for v in q))
        self.u0.append(tuple(float(v) for v in u))
        return len(self.mass) - 1

    def add_revolute(self, a, b, anchor_a, anchor_b, axis_b=(0, 1, 0),
                     perp1_a=(1, 0, 0), perp2_a=(0, 0, 1), axis_a=(0, 1, 0),
                     act=ACT_NONE, kp=0.0, kd=0.0) -> int:
        """Revolute joint: anchors coincide and axis_b stays normal to perp1_a, perp2_a.
        The joint angle (position servos) is that of R_b perp1_a from R_a perp1_a about
        R_a axis_a: zero where the two bodies' frames coincide."""
        self.joints.append(dict(a=a, b=b, anchor_a=anchor_a, anchor_b=anchor_b,
                                axis_b=axis_b, perp1_a=perp1_a, perp2_a=perp2_a,
                                axis_a=axis_a, act=act, kp=kp, kd=kd))
        return len(self.joints) - 1

    def add_slot(self, kind, a, local=(0, 0, 0), radius=0.0, mu=0.5, b=-1,
                 feature=-1, face_h=0.0, axis=(0.0, 0.0, 0.0)) -> int:
        """A contact proxy of body a: a sphere of `radius` at `local` (a point
        for radius 0), or, with a non-zero `axis` (body frame), the circle of
        that radius about `local` in the plane normal to the axis (a rim of a
        cylindrical wheel).  Rim circles touch static features only."""
        ax = np.asarray(axis, dtype=np.float64)
        na = float(np.linalg.norm(ax))
        if na > 0.0:
            if kind == SLOT_BODYFACE:
                raise ValueError("a rim circle touches static features only")
            if not radius > 0.0:
                raise ValueError("a rim circle needs a positive radius")
            ax = ax / na
        self.slots.append(dict(kind=kind, a=a, b=b, feature=feature, local=local,
                               radius=radius, mu=mu, face_h=face_h, axis=tuple(float(v) for v in ax)))
        return len(self.slots) - 1

    def add_obstacle(self, center, half) -> int:
        self.obstacles.append(tuple(center) + tuple(half))
        return len(self.obstacles) - 1

    @property
    def n_ctrl(self) -> int:
        return sum(1 for j in self.joints if j["act"] != ACT_NONE)

    @property
    def n_servo(self) -> int:
        return sum(1 for j in self.joints if j["act"] in (ACT_SERVO_VEL, ACT_TORQUE_DAMPED, ACT_SERVO_POS))

    @property
    def lam_len(self) -> int:
        return 5 * len(self.joints) + self.n_servo + 3 * len(self.slots)

    @property
    def row_cap(self) -> int:
        return 5 * len(self.joints) + self.n_servo + 3 * self.contact_cap


@dataclasses.dataclass
class Heightmap:
    """Regular-grid heightmap; cell (i, j) is split along its (i,j)-(i+1,j+1) diagonal."""
    n: int
    spacing: float
    origin: Sequence[float]
    heights: np.ndarray   # [n, n] heights, index [i (x), j (y)]


@dataclasses.dataclass
class Batch:
    """Flat world-major arrays describing W worlds (all int32 / float64)."""
    n_worlds: int
    body_off: np.ndarray
    body_mass: np.ndarray
    body_inertia: np.ndarray
    joint_off: np.ndarray
    joint_body: np.ndarray
    joint_frame: np.ndarray
    joint_act: np.ndarray
    joint_kp: np.ndarray
    joint_kd: np.ndarray
    ctrl_off: np.ndarray
    slot_off: np.ndarray
    slot_int: np.ndarray
    slot_real: np.ndarray
    obs_off: np.ndarray
    obs_box: np.ndarray
    lam_off: np.ndarray
    row_off: np.ndarray
    contact_cap: np.ndarray
    world_hmap: np.ndarray
    hmap_n: int
    hmap_spacing: float
    hmap_origin: np.ndarray
    hmap_heights: np.ndarray
    q0: np.ndarray
    u0: np.ndarray
    loss_body: np.ndarray
    target: np.ndarray
    worlds: List[World]

    @property
    def n_bodies(self):
        return int(self.body_off[-1])

    @property
    def n_lam(self):
        return int(self.lam_off[-1])

    @property
    def n_ctrl(self):
        return int(self.ctrl_off[-1])

    @property
    def n_slots(self):
        return int(self.slot_off[-1])

    def max_bodies(self):
        return int(np.max(np.diff(self.body_off))) if self.n_worlds else 0

    def max_rows(self):
        return int(np.max(np.diff(self.row_off))) if self.n_worlds else 0


def _offsets(counts):
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(np.asarray(counts, dtype=np.int64))
    return off


def pack(worlds: Sequence[World], heightmaps: Sequence[Heightmap] = ()) -> Batch:
    """Pack worlds into flat world-major arrays."""
    W = len(worlds)
    body_off = _offsets([len(w.mass) for w in worlds])
    joint_off = _offsets([len(w.joints) for w in worlds])
    ctrl_off = _offsets([w.n_ctrl for w in worlds])
    slot_off = _offsets([len(w.slots) for w in worlds])
    obs_off = _offsets([len(w.obstacles) for w in worlds])
    lam_off = _offsets([w.lam_len for w in worlds])
    row_off = _offsets([w.row_cap for w in worlds])

    def cat(rows, width, dtype):
        if not rows:
            return np.zeros((0, width), dtype=dtype)
        return np.ascontiguousarray(np.asarray(rows, dtype=dtype).reshape(-1, width))

    mass = np.array([m for w in worlds for m in w.mass], dtype=np.float64)
    inertia = cat([i for w in worlds for i in w.inertia], 3, np.float64)
    jb, jf, ja, jk, jd = [], [], [], [], []
    for w in worlds:
        for j in w.joints:
            jb.append((j["a"], j["b"]))
            jf.append(tuple(j["anchor_a"]) + tuple(j["anchor_b"]) + tuple(j["axis_b"]) +
                      tuple(j["perp1_a"]) + tuple(j["perp2_a"]) + tuple(j["axis_a"]))
            ja.append(j["act"])
            jk.append(j["kp"])
            jd.append(j.get("kd", 0.0))
    si, sr = [], []
    for w in worlds:
        for s in w.slots:
            si.append((s["kind"], s["a"], s["b"], s["feature"]))
            sr.append(tuple(s["local"]) + (s["radius"], s["mu"], s["face_h"]) + tuple(s.get("axis", (0.0, 0.0, 0.0))))
    obs = cat([o for w in worlds for o in w.obstacles], 6, np.float64)
    if heightmaps:
        n = heightmaps[0].n
        sp = heightmaps[0].spacing
        for hm in heightmaps:
            assert hm.n == n and hm.spacing == sp, "heightmaps of one batch share grid size"
        hmo = np.array([tuple(hm.origin)[:2] for hm in heightmaps], dtype=np.float64)
        hmh = np.ascontiguousarray(np.stack([hm.heights for hm in heightmaps]).astype(np.float64))
    else:
        n, sp = 0, 0.0
        hmo = np.zeros((0, 2), dtype=np.float64)
        hmh = np.zeros((0, 0, 0), dtype=np.float64)
    q0 = cat([q for w in worlds for q in w.q0], 7, np.float64)
    u0 = cat([u for w in worlds for u in w.u0], 6, np.float64)
    return Batch(
        n_worlds=W, body_off=body_off, body_mass=mass, body_inertia=inertia,
        joint_off=joint_off, joint_body=cat(jb, 2, np.int32), joint_frame=cat(jf, JOINT_FRAME_LEN, np.float64),
        joint_act=np.array(ja, dtype=np.int32), joint_kp=np.array(jk, dtype=np.float64),
        joint_kd=np.array(jd, dtype=np.float64), ctrl_off=ctrl_off, slot_off=slot_off, slot_int=cat(si, SLOT_INT_LEN, np.int32),
        slot_real=cat(sr, SLOT_REAL_LEN, np.float64), obs_off=obs_off, obs_box=obs,
        lam_off=lam_off, row_off=row_off,
        contact_cap=np.array([w.contact_cap for w in worlds], dtype=np.int32),
        world_hmap=np.array([w.heightmap for w in worlds], dtype=np.int32),
        hmap_n=int(n), hmap_spacing=float(sp), hmap_origin=hmo, hmap_heights=hmh,
        q0=q0, u0=u0,
        loss_body=np.array([w.loss_body for w in worlds], dtype=np.int32),
        target=cat([tuple(w.target) for w in worlds], 2, np.float64),
        worlds=list(worlds))


def world_rngs(seed: int, n: int):
    """One independent generator per world, reproducible for any batch size."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# --------------------------------------------------------------------------
# workload builders
# --------------------------------------------------------------------------

BOX_SIZE = (0.5, 0.3, 0.2)
BOX_MASS = 1.0
BOX_MU = 0.8


def box_world(rng=None, *, yaw=None, v=None, w=None, target=None, z=None, mu=BOX_MU,
              size=BOX_SIZE, mass=BOX_MASS) -> World:
    """Single box of 0.5 x 0.3 x 0.2 m, 1 kg, on the ground plane; 4 bottom-corner slots.

    With a generator, yaw ~ U(-pi, pi), v_xy ~ U(-2, 2), omega ~ N(0, 0.5),
    target ~ U(-1, 1)^2; explicit keyword values override the draws.
    """
    sx, sy, sz = size
    if rng is not None:
        yaw = rng.uniform(-math.pi, math.pi) if yaw is None else yaw
        vxy = rng.uniform(-2.0, 2.0, size=2)
        om = rng.normal(0.0, 0.5, size=3)
        tg = rng.uniform(-1.0, 1.0, size=2)
        v = (vxy[0], vxy[1], 0.0) if v is None else v
        w = tuple(om) if w is None else w
        target = tuple(tg) if target is None else target
    yaw = 0.0 if yaw is None else yaw
    v = (0.0, 0.0, 0.0) if v is None else v
    w = (0.0, 0.0, 0.0) if w is None else w
    target = (0.0, 0.0) if target is None else target
    z = 0.5 * sz if z is None else z
    wd = World(contact_cap=4)
    b = wd.add_body(mass, box_inertia(mass, sx, sy, sz), (0.0, 0.0, z) + yaw_quat(yaw), tuple(v) + tuple(w))
    for cx in (-0.5 * sx, 0.5 * sx):
        for cy in (-0.5 * sy, 0.5 * sy):
            wd.add_slot(SLOT_PLANE, b, local=(cx, cy, -0.5 * sz), mu=mu)
    wd.loss_body = b
    wd.target = target
    return wd


CHASSIS_SIZE = (0.6, 0.4, 0.15)
CHASSIS_MASS = 10.0
WHEEL_R = 0.1
WHEEL_W = 0.05
WHEEL_MASS = 0.5
WHEEL_POS = ((0.25, 0.23), (0.25, -0.23), (-0.25, 0.23), (-0.25, -0.23))
OBSTACLE_SIZE = (1.2, 0.8, 0.15)
ROBOT_MU = 1.0
ROBOT_KNOTS = 8
AXLE_DAMPING = 0.05    # N m s / rad: gain of the axle's zero-speed servo row


def robot_world(rng=None, *, yaw=0.0, obstacle_x=1.0, knots=None, mu=ROBOT_MU,
                servo_kp=None, with_obstacle=True, contact_cap=16,
                axle_damping=AXLE_DAMPING, obstacle_size=OBSTACLE_SIZE, wheels: str = "sphere") -> World:
    """Wheeled robot: 10 kg chassis box and four 0.5 kg wheels on revolute joints.

    The wheels are driven by torques (8 spline knots per wheel) with viscous
    axle damping expressed as the implicit servo row of the paper with a zero
    speed target (gain ``axle_damping``; 0 gives pure torque), or, with
    ``servo_kp``, by velocity servos.  Wheel contact uses a sphere proxy of the
    wheel radius at the wheel centre (rotation invariant about the axle), or
    with ``wheels="cylinder"`` the wheel's two rim circles (radius WHEEL_R,
    WHEEL_W apart, about the wheel's y axis); the chassis uses its 8 corners
    and 5 bottom-face points.  ``obstacle_x`` is the x of the obstacle's near
    face; the obstacle (``obstacle_size``, 1.2 x 0.8 x 0.15 m by default) is
    centred at y = 0.
    """
    if wheels not in ("cylinder", "sphere"):
        raise ValueError("wheels: 'cylinder' or 'sphere'")
    cx, cy, cz = CHASSIS_SIZE
    wd = World(contact_cap=contact_cap)
    zc = WHEEL_R
    qc = (0.0, 0.0, zc) + yaw_quat(yaw)
    c = wd.add_body(CHASSIS_MASS, box_inertia(CHASSIS_MASS, cx, cy, cz), qc)
    cyaw, syaw = math.cos(yaw), math.sin(yaw)
    wheel_bodies = []
    for (wx, wy) in WHEEL_POS:
        px, py = cyaw * wx - syaw * wy, syaw * wx + cyaw * wy
        wheel_bodies.append(wd.add_body(WHEEL_MASS, cylinder_inertia_y(WHEEL_MASS, WHEEL_R, WHEEL_W),
                                        (px, py, zc) + yaw_quat(yaw)))
    if servo_kp is not None:
        act, kp = ACT_SERVO_VEL, float(servo_kp)
    elif axle_damping:
        act, kp = ACT_TORQUE_DAMPED, float(axle_damping)
    else:
        act, kp = ACT_TORQUE, 0.0
    for b, (wx, wy) in zip(wheel_bodies, WHEEL_POS):
        wd.add_revolute(c, b, anchor_a=(wx, wy, 0.0), anchor_b=(0.0, 0.0, 0.0), act=act, kp=kp)
    kinds = [SLOT_PLANE] + ([SLOT_BOX] if with_obstacle else [])
    for b in wheel_bodies:
        for k in kinds:
            if wheels == "cylinder":
                for o in (-0.5 * WHEEL_W, 0.5 * WHEEL_W):
                    wd.add_slot(k, b, local=(0.0, o, 0.0), radius=WHEEL_R, mu=mu,
                                feature=0 if k == SLOT_BOX else -1, axis=(0.0, 1.0, 0.0))
            else:
                wd.add_slot(k, b, radius=WHEEL_R, mu=mu, feature=0 if k == SLOT_BOX else -1)
    pts = [(sx * 0.5 * cx, sy * 0.5 * cy, sz * 0.5 * cz)
           for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]
    pts += [(0.0, 0.0, -0.5 * cz), (0.5 * cx, 0.0, -0.5 * cz), (-0.5 * cx, 0.0, -0.5 * cz),
            (0.0, 0.5 * cy, -0.5 * cz), (0.0, -0.5 * cy, -0.5 * cz)]
    for p in pts:
        for k in kinds:
            wd.add_slot(k, c, local=p, mu=mu, feature=0 if k == SLOT_BOX else -1)
    if with_obstacle:
        ox, oy, oz = obstacle_size
        wd.add_obstacle((obstacle_x + 0.5 * ox, 0.0, 0.5 * oz), (0.5 * ox, 0.5 * oy, 0.5 * oz))
    if knots is None:
        knots = rng.uniform(-2.0, 2.0, size=(4, ROBOT_KNOTS)) if rng is not None \
            else np.zeros((4, ROBOT_KNOTS))
    wd.knots = np.asarray(knots, dtype=np.float64)
    wd.loss_body = c
    wd.target = (3.0, 0.0)
    return wd


def stack_world(rng, n_boxes: int) -> World:
    """Stack of n cubes (edge ~ U(0.1, 0.5), largest at the bottom), at rest.

    Masses ~ U(0.5, 5) kg, one mu ~ U(0.3, 1.2) per world, velocities
    ~ U(-0.05, 0.05) m/s.  Box 0 rests on the ground with its 4 bottom
    corners; box i > 0 rests its 4 bottom corners on the top face of box i-1,
    offset laterally so that the corners stay over that face.
    """
    edges = np.sort(rng.uniform(0.1, 0.5, size=n_boxes))[::-1]
    masses = rng.uniform(0.5, 5.0, size=n_boxes)
    mu = float(rng.uniform(0.3, 1.2))
    wd = World(contact_cap=4 * n_boxes)
    z = 0.0
    x = y = 0.0
    prev = None
    for i in range(n_boxes):
        e = float(edges[i])
        if prev is not None:
            slack = 0.5 * (float(edges[i - 1]) - e)
            x = prev[0] + rng.uniform(-0.5, 0.5) * slack
            y = prev[1] + rng.uniform(-0.5, 0.5) * slack
        z = z + (0.5 * float(edges[i - 1]) if i > 0 else 0.0) + 0.5 * e
        v = rng.uniform(-0.05, 0.05, size=3)
        b = wd.add_body(float(masses[i]), box_inertia(float(masses[i]), e, e, e),
                        (x, y, z, 0.0, 0.0, 0.0, 1.0), (v[0], v[1], v[2], 0.0, 0.0, 0.0))
        for sx in (-1, 1):
            for sy in (-1, 1):
                loc = (sx * 0.5 * e, sy * 0.5 * e, -0.5 * e)
                if i == 0:
                    wd.add_slot(SLOT_PLANE, b, local=loc, mu=mu)
                else:
                    wd.add_slot(SLOT_BODYFACE, b, local=loc, mu=mu, b=b - 1,
                                face_h=0.5 * float(edges[i - 1]))
        prev = (x, y)
    wd.loss_body = n_boxes - 1
    return wd


TERRAIN_N = 128          # vertices per side
TERRAIN_SPACING = 0.05   # m
TERRAIN_AMP = 0.3        # m, peak |height|
TERRAIN_ORIGIN = (-1.6, -0.5 * (TERRAIN_N - 1) * TERRAIN_SPACING)
TERRAIN_FEATURES = 4     # candidate mesh features per wheel proxy


def value_noise_heightmap(seed: int, n: int = TERRAIN_N, spacing: float = TERRAIN_SPACING,
                          origin=TERRAIN_ORIGIN, amp: float = TERRAIN_AMP,
                          lattices=(1.6, 0.8, 0.4, 0.2)) -> Heightmap:
    """Four-octave value noise: lattice values U(-1, 1) on grids of the given
    spacings, smoothstep-bilinear interpolation, octave o weighted 0.5**o, the
    sum scaled so that its peak |height| is `amp`."""
    rng = np.random.default_rng(seed)
    xs = origin[0] + spacing * np.arange(n)
    ys = origin[1] + spacing * np.arange(n)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    H = np.zeros((n, n))
    for o, L in enumerate(lattices):
        gx = int(np.ceil((xs[-1] - xs[0]) / L)) + 2
        gy = int(np.ceil((ys[-1] - ys[0]) / L)) + 2
        val = rng.uniform(-1.0, 1.0, size=(gx, gy))
        u = (X - xs[0]) / L
        v = (Y - ys[0]) / L
        i0 = np.floor(u).astype(int)
        j0 = np.floor(v).astype(int)
        fu = u - i0
        fv = v - j0
        su = fu * fu * (3 - 2 * fu)
        sv = fv * fv * (3 - 2 * fv)
        a = val[i0, j0] * (1 - su) + val[i0 + 1, j0] * su
        b = val[i0, j0 + 1] * (1 - su) + val[i0 + 1, j0 + 1] * su
        H += (0.5 ** o) * (a * (1 - sv) + b * sv)
    H *= amp / np.max(np.abs(H))
    return Heightmap(n=n, spacing=spacing, origin=tuple(origin), heights=np.ascontiguousarray(H))


def terrain_height(hm: Heightmap, x: float, y: float) -> float:
    """Height of the triangulated heightmap at (x, y) (cells cut along (i,j)-(i+1,j+1))."""
    u = (x - hm.origin[0]) / hm.spacing
    v = (y - hm.origin[1]) / hm.spacing
    i = int(min(max(np.floor(u), 0), hm.n - 2))
    j = int(min(max(np.floor(v), 0), hm.n - 2))
    fu, fv = u - i, v - j
    H = hm.heights
    if fu >= fv:   # triangle (i,j), (i+1,j), (i+1,j+1)
        return float(H[i, j] + fu * (H[i + 1, j] - H[i, j]) + fv * (H[i + 1, j + 1] - H[i + 1, j]))
    return float(H[i, j] + fv * (H[i, j + 1] - H[i, j]) + fu * (H[i + 1, j + 1] - H[i, j + 1]))


def robot_terrain_world(rng=None, hm: Heightmap = None, hmap_index: int = 0, *, yaw=0.0, knots=None,
                        mu=ROBOT_MU, n_feat: int = TERRAIN_FEATURES, contact_cap=24,
                        axle_damping=AXLE_DAMPING, start=(0.0, 0.0), wheels: str = "cylinder") -> World:
    """The wheeled robot on heightmap terrain, placed at `start` with its
    wheels just above the surface.  Cylindrical wheels (the default; radius
    WHEEL_R, width WHEEL_W, axis the wheel body's y axis) touch the mesh with
    their two rim circles, each with n_feat terrain slots (its nearest
    candidate mesh features); with wheels="sphere" each wheel is one sphere of
    the wheel radius with n_feat slots.  Each chassis point has one slot."""
    if wheels not in ("cylinder", "sphere"):
        raise ValueError("wheels: 'cylinder' or 'sphere'")
    cx, cy, cz = CHASSIS_SIZE
    wd = World(contact_cap=contact_cap)
    cyaw, syaw = math.cos(yaw), math.sin(yaw)
    wxy = [(start[0] + cyaw * wx - syaw * wy, start[1] + syaw * wx + cyaw * wy) for (wx, wy) in WHEEL_POS]
    rims = (-0.5 * WHEEL_W, 0.5 * WHEEL_W) if wheels == "cylinder" else (0.0,)
    # clear the surface under the wheels' rims and under the chassis bottom (sampled every 5 cm)
    zc = 0.0
    if hm is not None:
        zc = max(terrain_height(hm, x - syaw * o, y + cyaw * o) + WHEEL_R for (x, y) in wxy for o in rims)
        for sx in np.linspace(-0.5 * cx, 0.5 * cx, 13):
            for sy in np.linspace(-0.5 * cy, 0.5 * cy, 9):
                x = start[0] + cyaw * sx - syaw * sy
                y = start[1] + syaw * sx + cyaw * sy
                zc = max(zc, terrain_height(hm, x, y) + 0.5 * cz)
    zc += 1e-3
    c = wd.add_body(CHASSIS_MASS, box_inertia(CHASSIS_MASS, cx, cy, cz), (start[0], start[1], zc) + yaw_quat(yaw))
    wheel_bodies = [wd.add_body(WHEEL_MASS, cylinder_inertia_y(WHEEL_MASS, WHEEL_R, WHEEL_W),
                                (px, py, zc) + yaw_quat(yaw)) for (px, py) in wxy]
    act, kp = (ACT_TORQUE_DAMPED, float(axle_damping)) if axle_damping else (ACT_TORQUE, 0.0)
    for b, (wx, wy) in zip(wheel_bodies, WHEEL_POS):
        wd.add_revolute(c, b, anchor_a=(wx, wy, 0.0), anchor_b=(0.0, 0.0, 0.0), act=act, kp=kp)
    for b in wheel_bodies:
        for o in rims:
            for k in range(n_feat):
                if wheels == "cylinder":
                    wd.add_slot(SLOT_HEIGHTMAP, b, local=(0.0, o, 0.0), radius=WHEEL_R, mu=mu, feature=k,
                                axis=(0.0, 1.0, 0.0))
                else:
                    wd.add_slot(SLOT_HEIGHTMAP, b, radius=WHEEL_R, mu=mu, feature=k)
    pts = [(sx * 0.5 * cx, sy * 0.5 * cy, sz * 0.5 * cz)
           for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]
    pts += [(0.0, 0.0, -0.5 * cz), (0.5 * cx, 0.0, -0.5 * cz), (-0.5 * cx, 0.0, -0.5 * cz),
            (0.0, 0.5 * cy, -0.5 * cz), (0.0, -0.5 * cy, -0.5 * cz)]
    for p in pts:
        wd.add_slot(SLOT_HEIGHTMAP, c, local=p, mu=mu, feature=0)
    if knots is None:
        knots = rng.uniform(-2.0, 2.0, size=(4, ROBOT_KNOTS)) if rng is not None \
            else np.zeros((4, ROBOT_KNOTS))
    wd.knots = np.asarray(knots, dtype=np.float64)
    wd.heightmap = hmap_index
    wd.loss_body = c
    wd.target = (3.0, 0.0)
    return wd


def terrain_batch(n_worlds: int, seed: int = 0, n_maps: int = 1, n: int = TERRAIN_N,
                  wheels: str = "cylinder") -> Batch:
    """Robots on n_maps value-noise terrains (world w on map w % n_maps)."""
    maps = [value_noise_heightmap(seed * 1000 + k, n=n) for k in range(n_maps)]
    worlds = []
    for w, r in enumerate(world_rngs(seed, n_worlds)):
        k = w % n_maps
        worlds.append(robot_terrain_world(r, maps[k], k, yaw=float(r.uniform(-0.3, 0.3)), wheels=wheels))
    return pack(worlds, maps)


def terrain_request_batch(seed: int, n_worlds: int, wheels: str = "cylinder") -> Batch:
    """One trajectory-optimisation request: n_worlds robots (seeded yaw and
    knots) on the request's own value-noise terrain (heightmap index 0)."""
    hm = value_noise_heightmap(10_000 + seed)
    worlds = [robot_terrain_world(r, hm, 0, yaw=float(r.uniform(-0.3, 0.3)), wheels=wheels)
              for r in world_rngs(seed, n_worlds)]
    return pack(worlds, [hm])


def box_batch(n_worlds: int, seed: int = 0) -> Batch:
    return pack([box_world(r) for r in world_rngs(seed, n_worlds)])


def robot_batch(n_worlds: int, seed: int = 0, *, randomize=True) -> Batch:
    """Robot worlds; with ``randomize`` yaw ~ U(-0.3, 0.3), obstacle x ~ U(0.8, 1.4)."""
    worlds = []
    for r in world_rngs(seed, n_worlds):
        if randomize:
            knots = r.uniform(-2.0, 2.0, size=(4, ROBOT_KNOTS))
            yaw = float(r.uniform(-0.3, 0.3))
            ox = float(r.uniform(0.8, 1.4))
            worlds.append(robot_world(knots=knots, yaw=yaw, obstacle_x=ox))
        else:
            worlds.append(robot_world(r))
    return pack(worlds)


def mixed_batch(n_stacks: int, n_robots: int, seed: int = 0, max_boxes: int = 32) -> Batch:
    """Uneven batch: box stacks of 1..max_boxes boxes followed by robots."""
    rngs = world_rngs(seed, n_stacks + n_robots)
    worlds = []
    for r in rngs[:n_stacks]:
        worlds.append(stack_world(r, int(r.integers(1, max_boxes + 1))))
    for r in rngs[n_stacks:]:
        knots = r.uniform(-2.0, 2.0, size=(4, ROBOT_KNOTS))
        worlds.append(robot_world(knots=knots, yaw=float(r.uniform(-0.3, 0.3)),
                                  obstacle_x=float(r.uniform(0.8, 1.4))))
    return pack(worlds)


def knots_array(batch: Batch, K: int) -> np.ndarray:
    """Per-world control knots packed as [n_ctrl_total, K] (zeros where absent)."""
    out = np.zeros((batch.n_ctrl, K), dtype=np.float64)
    for wi, w in enumerate(batch.worlds):
        n = w.n_ctrl
        if n and w.knots is not None:
            out[batch.ctrl_off[wi]:batch.ctrl_off[wi] + n, :] = w.knots[:, :K]
    return out


def solver_params(**over) -> dict:
    """Step parameters shared by both implementations (a plain dictionary).

    h: step (s); tol: Newton tolerance on the residual norm; k_max / k_min:
    iteration budget and best-iterate floor; eps: smoothing of the FB function
    and of norms; delta_g: guard of denominators; delta_reg: relative Schur
    diagonal regularisation of the Newton iterations; delta_reg_adj: that of the
    adjoint's system (the factor the adjoint solves with); delta0: contact
    activation margin (m);
    sigma_mode: 1 scales the FB multiplier argument by the Delassus diagonal,
    0 keeps the literal unit scale; n_feat: heightmap features per proxy;
    newton_mode: 0 uses the generalized Jacobian of the constraint rows, 1
    freezes the friction weight W within an iteration (symmetric Schur matrix);
    ls_max: step halvings of the residual-decrease step length (0: full steps);
    refine: most operator applications of the adjoint's Krylov solve of the
    exact implicit-function Jacobian (0: the stored factor's solve alone);
    truncate: 1 treats the contact geometry as a constant of each step in the
    adjoint's q- pull-back (the truncated pull-back of long terrain horizons);
    linear_solver: the Newton step's solve, 0 the banded LU of the Schur matrix, 1 a
    matrix-free Krylov solve of at most krylov_iters products (the oracle always
    solves exactly: the root, not the path, is compared).
    """
    p = dict(h=0.1, gravity=GRAVITY, tol=1e-10, k_max=16, k_min=4, eps=1e-8,
             delta_g=1e-12, delta_reg=1e-6, delta_reg_adj=1e-8, delta0=0.02, sigma_mode=1, n_feat=4,
             newton_mode=0, ls_max=4, refine=8, truncate=0,
             linear_solver=0, krylov_iters=16)
    p.update(over)
    return p
