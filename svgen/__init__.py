"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no kinematics, no distances, no network evaluation).  Every
floating-point value it returns is exactly representable in FP32, so the FP32 GPU
path and the FP64 oracle start from bit-identical inputs.

Recipes (the paper gives no robot data, no scene files and no weights, so these
are synthetic stand-ins for its workloads):

* ``make_arm``: a 6-DOF serial arm in standard DH form with 7 capsules.  Capsule
  k (k = 1..6) spans from the origin of frame k-1 to the origin of frame k;
  capsule 7 is a tool along the z axis of the last frame.  Each capsule endpoint
  is stated as (frame index, point in that frame), so the description needs no
  kinematics to write down.
* ``make_motions``: start/goal configurations drawn uniformly within the joint
  limits, as in the paper's dataset generation (Sec. IV-C); spline motions add
  two via configurations drawn the same way.
* ``bin_cloud``: points on the five walls of an open bin plus the exposed faces
  of random boxes resting on its floor, area proportional, with Gaussian noise.
  It stands in for the proprietary bin-picking clouds of Sec. V-C.
* ``uniform_cube``: points uniform in an axis-aligned cube around the base.
* ``mlp_init``: the flat FP32 parameter vector of a plain softplus MLP,
  uniform(+-1/sqrt(fan_in)) per layer, weights then bias.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DOF = 6
N_CAPS = 7


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(x):
    """Round to FP32 and return float64 values that are exactly FP32-representable."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclass
class Arm:
    """Serial arm: standard DH rows (a, alpha, d, theta_offset), joint limits, capsules.

    ``cap_frame[k] = (fa, fb)`` are the frames of capsule k's two endpoints
    (0 = base frame, i = frame after joint i); ``cap_p[k] = (pa, pb)`` their
    coordinates in those frames (metres); ``cap_r[k]`` the radius.
    """
    dh: np.ndarray                 # [dof][4] float64 (FP32-exact)
    qlim: np.ndarray               # [dof][2] float64 (FP32-exact)
    cap_frame: np.ndarray          # [K][2] int32
    cap_p: np.ndarray              # [K][2][3] float64 (FP32-exact)
    cap_r: np.ndarray              # [K] float64 (FP32-exact)
    seed: int = 0

    @property
    def dof(self) -> int:
        return int(self.dh.shape[0])

    @property
    def n_caps(self) -> int:
        return int(self.cap_r.shape[0])


def make_arm(seed: int) -> Arm:
    """Synthetic 6-DOF arm: link lengths 0.1-0.5 m, limits +-170 deg, 7 capsules r 0.03-0.08 m.

    Fixed draw order (PCG64(seed)): per joint k=1..6: length, elevation angle phi,
    twist choice; then the tool length; then 7 radii.  a_k = l cos(phi),
    d_k = l sin(phi), alpha_k in {-pi/2, 0, +pi/2}, theta_offset = 0.
    """
    g = _rng(seed)
    dh = np.zeros((DOF, 4))
    for k in range(DOF):
        ln = g.uniform(0.1, 0.5)
        phi = g.uniform(0.0, math.pi / 2)
        alpha = (-math.pi / 2, 0.0, math.pi / 2)[int(g.integers(0, 3))]
        dh[k] = (ln * math.cos(phi), alpha, ln * math.sin(phi), 0.0)
    tool = g.uniform(0.1, 0.5)
    radii = g.uniform(0.03, 0.08, size=N_CAPS)
    lim = 170.0 * math.pi / 180.0
    qlim = np.tile(np.array([-lim, lim]), (DOF, 1))
    cap_frame = np.zeros((N_CAPS, 2), np.int32)
    cap_p = np.zeros((N_CAPS, 2, 3))
    for k in range(DOF):
        cap_frame[k] = (k, k + 1)          # origin of frame k -> origin of frame k+1
    cap_frame[DOF] = (DOF, DOF)
    cap_p[DOF, 1] = (0.0, 0.0, tool)       # tool along the last frame's z axis
    return Arm(dh=_f32(dh), qlim=_f32(qlim), cap_frame=cap_frame, cap_p=_f32(cap_p),
               cap_r=_f32(radii), seed=seed)


@dataclass
class Motions:
    """A batch of motions: type 'linear' or 'spline', T samples, q0/q1 [M][dof], via [M][2][dof]."""
    q0: np.ndarray
    q1: np.ndarray
    T: int
    kind: str = "linear"
    via: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.q0.shape[0])


def make_motions(arm: Arm, n: int, T: int, seed: int, kind: str = "linear") -> Motions:
    """q0, q1 (and two vias for splines) uniform within the joint limits, FP32-exact."""
    g = _rng(seed)
    lo, hi = arm.qlim[:, 0], arm.qlim[:, 1]
    q0 = _f32(g.uniform(lo, hi, size=(n, arm.dof)))
    q1 = _f32(g.uniform(lo, hi, size=(n, arm.dof)))
    via = None
    if kind == "spline":
        via = _f32(g.uniform(lo, hi, size=(n, 2, arm.dof)))
    elif kind != "linear":
        raise ValueError(kind)
    return Motions(q0=q0, q1=q1, T=int(T), kind=kind, via=via)


def uniform_cube(n: int, seed: int, half: float = 0.6) -> np.ndarray:
    """n points uniform in [-half, half]^3, returned [n][3] float64 (FP32-exact)."""
    return _f32(_rng(seed).uniform(-half, half, size=(n, 3)))


# Bin placement: interior x in [0.15, 0.55], y in [-0.3, 0.3], floor z = -0.45, rim z = -0.15
BIN_X = (0.15, 0.55)
BIN_Y = (-0.3, 0.3)
BIN_Z = (-0.45, -0.15)


def _faces_of_bin():
    (x0, x1), (y0, y1), (z0, z1) = BIN_X, BIN_Y, BIN_Z
    o = np.array
    return [
        (o([x0, y0, z0]), o([x1 - x0, 0, 0]), o([0, y1 - y0, 0])),       # floor
        (o([x0, y0, z0]), o([0, y1 - y0, 0]), o([0, 0, z1 - z0])),       # wall x = x0
        (o([x1, y0, z0]), o([0, y1 - y0, 0]), o([0, 0, z1 - z0])),       # wall x = x1
        (o([x0, y0, z0]), o([x1 - x0, 0, 0]), o([0, 0, z1 - z0])),       # wall y = y0
        (o([x0, y1, z0]), o([x1 - x0, 0, 0]), o([0, 0, z1 - z0])),       # wall y = y1
    ]


def bin_cloud(n: int, seed: int, n_boxes: int = 30, box_lo: float = 0.03,
              box_hi: float = 0.15, sigma: float = 0.002) -> np.ndarray:
    """Bin-picking-shaped cloud of exactly n points, [n][3] float64 (FP32-exact).

    Faces: the 5 walls of the bin and, for each box (sides U[box_lo, box_hi]^3,
    random yaw, resting on the floor, centre uniform in the bin footprint), its
    top and 4 side faces.  Points are spread over the faces in proportion to
    area (multinomial), uniform within a face, then i.i.d. N(0, sigma^2) noise
    per coordinate is added.
    """
    g = _rng(seed)
    faces = _faces_of_bin()
    for _ in range(n_boxes):
        sx, sy, sz = g.uniform(box_lo, box_hi, size=3)
        yaw = g.uniform(0.0, 2 * math.pi)
        cx = g.uniform(*BIN_X)
        cy = g.uniform(*BIN_Y)
        c, s = math.cos(yaw), math.sin(yaw)
        ex = np.array([c, s, 0.0]) * sx          # box edge vectors in the world
        ey = np.array([-s, c, 0.0]) * sy
        ez = np.array([0.0, 0.0, sz])
        base = np.array([cx, cy, BIN_Z[0]]) - 0.5 * ex - 0.5 * ey
        faces += [
            (base + ez, ex, ey),                   # top
            (base, ex, ez), (base + ey, ex, ez),   # sides along x
            (base, ey, ez), (base + ex, ey, ez),   # sides along y
        ]
    area = np.array([np.linalg.norm(np.cross(u, v)) for _, u, v in faces])
    counts = g.multinomial(n, area / area.sum())
    pts = np.empty((n, 3))
    i = 0
    for (o, u, v), cnt in zip(faces, counts):
        ab = g.uniform(0.0, 1.0, size=(cnt, 2))
        pts[i:i + cnt] = o + ab[:, :1] * u + ab[:, 1:] * v
        i += cnt
    pts = pts[g.permutation(n)]
    pts += g.normal(0.0, sigma, size=pts.shape)
    return _f32(pts)


@dataclass
class MLPSpec:
    in_dim: int
    width: int
    n_hidden: int

    @property
    def n_params(self) -> int:
        w, n = self.width, self.n_hidden
        return (self.in_dim * w + w) + (n - 1) * (w * w + w) + (w + 1)

    def layer_shapes(self):
        """[(out, in)] for every linear layer, input layer first, output layer last."""
        w = self.width
        return [(w, self.in_dim)] + [(w, w)] * (self.n_hidden - 1) + [(1, w)]


def mlp_init(spec: MLPSpec, seed: int) -> np.ndarray:
    """Flat FP32 parameter vector: for each layer W (row-major [out][in]) then b.

    Values are uniform in +-1/sqrt(fan_in), drawn layer by layer, W before b.
    """
    g = _rng(seed)
    parts = []
    for out, fin in spec.layer_shapes():
        bound = 1.0 / math.sqrt(fin)
        parts.append(g.uniform(-bound, bound, size=out * fin))
        parts.append(g.uniform(-bound, bound, size=out))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == spec.n_params
    return flat


@dataclass(frozen=True)
class ResSpec:
    """The residual network's sizes: n_blocks blocks of dimension width."""
    in_dim: int
    width: int
    n_blocks: int

    @property
    def n_params(self) -> int:
        w, i = self.width, self.in_dim
        return (w * i + w) + self.n_blocks * (w * w + w * i + 5 * w) + (w + 1)


def res_init(spec: ResSpec, seed: int) -> np.ndarray:
    """Flat FP32 parameters of the residual network, in the order of its layout.

    Linear layers: uniform in +-1/sqrt(fan_in) (a block's fan_in is width + in_dim),
    W before b.  BatchNorm running statistics and affine terms as a trained layer might
    hold them: gamma U[0.8, 1.2], beta U[-0.1, 0.1], mu U[0, 0.5] (inputs are ReLU
    outputs), var U[0.5, 1.5].
    """
    g = _rng(seed)
    w, i = spec.width, spec.in_dim
    b0 = 1.0 / math.sqrt(i)
    parts = [g.uniform(-b0, b0, size=w * i), g.uniform(-b0, b0, size=w)]
    bb = 1.0 / math.sqrt(w + i)
    for _ in range(spec.n_blocks):
        parts += [g.uniform(-bb, bb, size=w * w), g.uniform(-bb, bb, size=w * i), g.uniform(-bb, bb, size=w),
                  g.uniform(0.8, 1.2, size=w), g.uniform(-0.1, 0.1, size=w), g.uniform(0.0, 0.5, size=w),
                  g.uniform(0.5, 1.5, size=w)]
    bo = 1.0 / math.sqrt(w)
    parts += [g.uniform(-bo, bo, size=w), g.uniform(-bo, bo, size=1)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == spec.n_params
    return flat


def uniforms(seed: int, rows: int, cols: int) -> np.ndarray:
    """[rows][cols] float32 numbers uniform in [0, 1) (strictly below 1 after rounding)."""
    u = _rng(seed).random((rows, cols), dtype=np.float32)
    return np.minimum(u, np.float32(1.0) - np.float32(2.0 ** -24))


def permutation(seed: int, n: int) -> np.ndarray:
    """A seeded permutation of range(n) as int32 (e.g. the sample order of one epoch)."""
    return _rng(seed).permutation(n).astype(np.int32)


def log_uniform_int(g: np.random.Generator, lo: int, hi: int) -> int:
    """round(exp(U(ln lo, ln hi))) clipped to [lo, hi]."""
    v = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    return min(max(v, lo), hi)


@dataclass
class Request:
    motions: Motions
    cloud: np.ndarray


def make_requests(arm: Arm, n_req: int, seed: int, m_range=(1, 2048), n_range=(2000, 200000),
                  T: int = 512, kind: str = "spline") -> list:
    """Uneven request mix: per request, motion count and cloud size drawn log-uniformly."""
    g = _rng(seed)
    reqs = []
    for r in range(n_req):
        m = log_uniform_int(g, *m_range)
        npts = log_uniform_int(g, *n_range)
        sub = int(g.integers(0, 2**31 - 1))
        reqs.append(Request(make_motions(arm, m, T, sub, kind), bin_cloud(npts, sub + 1)))
    return reqs


def _random_rotation(g: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix (from a normalised Gaussian quaternion)."""
    w, x, y, z = _unit4(g)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _unit4(g: np.random.Generator):
    q = g.normal(size=4)
    return q / np.linalg.norm(q)


def box_world(seed: int, n_boxes: int = 50, side=(0.01, 0.10), density: float = 1000.0,
              region=((-1.0, 1.0), (-1.0, 1.0), (0.0, 1.5))) -> np.ndarray:
    """Box-world cloud [n][3] (FP32-exact): points on the surfaces of n_boxes boxes.

    Boxes: sides U[side]^3, a uniformly random orientation, centre uniform in the
    region (the scenes of the paper's box-world experiment, Sec. V-B).  Points: density
    per square metre of surface (0.1 per cm^2 = 1000 per m^2), spread over all faces in
    proportion to area, uniform within a face.
    """
    g = _rng(seed)
    faces = []
    for _ in range(n_boxes):
        s = g.uniform(side[0], side[1], size=3)
        R = _random_rotation(g)
        c = np.array([g.uniform(*region[0]), g.uniform(*region[1]), g.uniform(*region[2])])
        e = [R[:, i] * s[i] for i in range(3)]                      # edge vectors
        corner = c - 0.5 * (e[0] + e[1] + e[2])
        for i, j, k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            faces.append((corner, e[i], e[j]))
            faces.append((corner + e[k], e[i], e[j]))
    area = np.array([np.linalg.norm(np.cross(u, v)) for _, u, v in faces])
    n = int(round(area.sum() * density))
    counts = g.multinomial(n, area / area.sum())
    pts = np.empty((n, 3))
    i = 0
    for (o, u, v), cnt in zip(faces, counts):
        ab = g.uniform(0.0, 1.0, size=(cnt, 2))
        pts[i:i + cnt] = o + ab[:, :1] * u + ab[:, 1:] * v
        i += cnt
    return _f32(pts[g.permutation(n)])


def scene_motions(arm: Arm, n_goals: int, T: int, seed: int) -> Motions:
    """One start configuration and n_goals goal configurations, uniform within the joint
    limits: the linear motions start -> goal_j of one scene (Sec. V-B)."""
    g = _rng(seed)
    lo, hi = arm.qlim[:, 0], arm.qlim[:, 1]
    q0 = _f32(g.uniform(lo, hi, size=(1, arm.dof)))
    q1 = _f32(g.uniform(lo, hi, size=(n_goals, arm.dof)))
    return Motions(q0=np.repeat(q0, n_goals, axis=0), q1=q1, T=int(T))


# Named workloads (seeds explicit).  Sizes follow the workloads of the paper's
# Sec. V as scaled up for a bin-picking batch on one GPU.
WORKLOADS = {
    "tiny": dict(arm_seed=1, motion_seed=11, n_motions=1, T=64, cloud="cube", n_points=4096,
                 cloud_seed=21, mlp=(15, 256, 4), mlp_seed=31),
    "bin20k": dict(arm_seed=1, motion_seed=12, n_motions=512, T=256, cloud="bin", n_points=20000,
                   cloud_seed=22, eps=0.01, tau=0.03, mlp=(15, 512, 8), mlp_seed=32),
    # the box-world scenes of Sec. V-B (50 boxes of 1-10 cm, 0.1 points per cm^2, one start
    # and 100 goals per scene, T = 200, eps = 5 mm) with the box region scaled by 1.2 to
    # this arm's reach; a 5 x 512 network as in that experiment
    "boxworld": dict(arm_seed=1, scenes=100, n_goals=100, T=200, eps=0.005, region_scale=1.2, scene_seed=300,
                     mlp=(15, 512, 5), mlp_seed=33, cube_half=1.8),
}


def box_world_scene(arm: Arm, scene: int, w: dict = None):
    """(motions, cloud) of box-world scene number `scene` of the named workload."""
    w = w or WORKLOADS["boxworld"]
    k = w["region_scale"]
    region = ((-k, k), (-k, k), (0.0, 1.5 * k))
    pts = box_world(w["scene_seed"] + 2 * scene, region=region)
    return scene_motions(arm, w["n_goals"], w["T"], w["scene_seed"] + 2 * scene + 1), pts
