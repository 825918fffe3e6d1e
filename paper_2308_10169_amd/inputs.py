"""Seeded synthetic workloads for the SEPSO planner.

This module only *generates inputs* (maps, obstacle motion, swarm settings);
it holds none of the method's arithmetic, so both the HIP path and the FP64
oracle can be fed from it.  Every coordinate, velocity and constant it emits
is exactly representable in FP32 (map geometry lies on a 1/256 grid), so the
two sides start from bit-identical inputs.

The paper's own obstacle layout exists only in figures that are not
available, so the maps are random stand-ins with the paper's shapes: a
366 x 366 map with static and moving rectangular obstacles, a moving start
and target (Sec. "Experiments Result on Path Planning"), and the constants of
Tables hyper1, hyper8, hyper8path and params_path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GRID = 256.0  # geometry lives on multiples of 1/256

# Table hyper8: DTPSO / H-SEPSO defaults, rows = groups,
# columns = C1, C2, C3, w_init, w_end, V_limit.
HYPER8 = np.array([
    [2, 1, 1, 0.4, 0.2, 0.2],
    [1, 1, 2, 0.7, 0.3, 0.1],
    [2, 2, 1, 0.8, 0.1, 0.6],
    [2, 2, 1, 0.8, 0.6, 0.4],
    [2, 1, 2, 0.2, 0.1, 0.3],
    [2, 1, 2, 0.9, 0.5, 0.5],
    [1, 2, 2, 0.4, 0.1, 0.8],
    [1, 2, 2, 0.9, 0.3, 0.3],
], dtype=np.float64)

# Table hyper8path: evolved L-SEPSO hyper-parameters for path planning.
HYPER8PATH = np.array([
    [1.53, 1.29, 1.34, 0.48, 0.19, 0.35],
    [1.72, 1.53, 1.34, 0.73, 0.28, 0.32],
    [1.34, 1.42, 1.33, 0.48, 0.21, 0.62],
    [1.76, 1.60, 1.21, 0.47, 0.30, 0.63],
    [1.68, 1.27, 1.25, 0.73, 0.36, 0.41],
    [1.66, 1.54, 1.54, 0.39, 0.16, 0.45],
    [1.57, 1.48, 1.75, 0.56, 0.34, 0.38],
    [1.31, 1.71, 1.23, 0.36, 0.25, 0.50],
], dtype=np.float64)

# Table hyper1 (plain PSO): C1 = C2 = 2, w 0.9 -> 0.4, V_limit 0.5; no Tbest term.
HYPER1_ROW = np.array([2.0, 2.0, 0.0, 0.9, 0.4, 0.5])

# Table params_path: penalty alpha, beta; PI fraction gamma; AT delta and window.
PARAMS_PATH = dict(alpha=30.0, beta=4, gamma=0.25, delta=10.0, tw=20)


def f32(x):
    """Round to the nearest FP32 value, returned as float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def snap(x):
    """Snap to the 1/256 grid."""
    return np.round(np.asarray(x, dtype=np.float64) * GRID) / GRID


@dataclasses.dataclass
class MapSpec:
    width: float
    height: float
    poly_ptr: np.ndarray      # int32, n_polys + 1
    verts: np.ndarray         # float64 (n_vert, 2), on the 1/256 grid
    start: np.ndarray         # float64 (2,)
    target: np.ndarray        # float64 (2,)
    poly_vel: np.ndarray      # float64 (n_polys, 2) cells / frame (0 = static)
    endpoint_vel: np.ndarray  # float64 (4,) start (vx, vy), target (vx, vy)

    @property
    def n_polys(self) -> int:
        return len(self.poly_ptr) - 1

    @property
    def n_edges(self) -> int:
        return int(self.poly_ptr[-1])

    @property
    def scale(self) -> float:
        return max(self.width, self.height)

    def copy(self) -> "MapSpec":
        return MapSpec(self.width, self.height, self.poly_ptr.copy(), self.verts.copy(),
                       self.start.copy(), self.target.copy(), self.poly_vel.copy(),
                       self.endpoint_vel.copy())


@dataclasses.dataclass
class SwarmSpec:
    groups: int
    particles: int
    waypoints: int
    max_iters: int
    hyper: np.ndarray         # (G, 6) float64, FP32-exact
    alpha: float
    beta: int
    seed: int = 0
    instance: int = 0
    use_pi: int = 0
    pi_gamma: float = 0.25
    pi_radius: float = 0.0
    at_mode: int = 0
    at_window: int = 5
    at_delta: float = 1e-3
    hsef_every: int = 0
    hsef_hyper: np.ndarray | None = None
    rand_per_dim: int = 0     # variant: one (r1, r2, r3) per coordinate instead of per particle

    def __post_init__(self):
        self.hyper = f32(self.hyper).reshape(self.groups, 6)
        self.alpha = float(f32(self.alpha))
        self.pi_gamma = float(f32(self.pi_gamma))
        self.pi_radius = float(f32(self.pi_radius))
        self.at_delta = float(f32(self.at_delta))
        if self.hsef_hyper is None:
            self.hsef_hyper = HYPER8[np.arange(self.groups) % 8]
        self.hsef_hyper = f32(self.hsef_hyper).reshape(self.groups, 6)


def _inside(box, pt, margin):
    x0, y0, w, h = box
    return (x0 - margin <= pt[0] <= x0 + w + margin) and (y0 - margin <= pt[1] <= y0 + h + margin)


def random_rects(rng, width, height, n, side_lo, side_hi, avoid=(), margin=1.0):
    """n axis-aligned rectangles: sides ~ U[side_lo, side_hi], lower-left
    corner uniform so the box lies in the map; boxes containing a point of
    `avoid` (with margin) are redrawn.  Returns (n, 4, 2) corner arrays."""
    out = []
    while len(out) < n:
        w, h = snap(rng.uniform(side_lo, side_hi, size=2))
        x0 = snap(rng.uniform(0.0, width - w))
        y0 = snap(rng.uniform(0.0, height - h))
        if any(_inside((x0, y0, w, h), p, margin) for p in avoid):
            continue
        out.append(np.array([[x0, y0], [x0 + w, y0], [x0 + w, y0 + h], [x0, y0 + h]]))
    return np.array(out, dtype=np.float64).reshape(n, 4, 2)


def random_quads(rng, width, height, n, ax_lo, ax_hi):
    """n convex quadrilaterals: four sorted random angles on an ellipse with
    random semi-axes, centred uniformly inside the map."""
    out = []
    for _ in range(n):
        a, b = rng.uniform(ax_lo, ax_hi, size=2)
        cx = rng.uniform(a, width - a)
        cy = rng.uniform(b, height - b)
        th = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=4))
        q = np.stack([cx + a * np.cos(th), cy + b * np.sin(th)], axis=1)
        q = np.clip(snap(q), 0.0, [width, height])
        out.append(q)
    return np.array(out, dtype=np.float64).reshape(n, 4, 2)


def random_stars(rng, width, height, n, r_lo, r_hi, spikes=(5, 8)):
    """n non-convex star polygons: 2m vertices alternating between an outer
    radius ~ U[r_lo, r_hi] and 0.4 of it, jittered angles, centred inside the
    map (simple polygons, counter-clockwise)."""
    out = []
    for _ in range(n):
        m = int(rng.integers(spikes[0], spikes[1] + 1))
        ro = rng.uniform(r_lo, r_hi)
        cx, cy = rng.uniform(ro, width - ro), rng.uniform(ro, height - ro)
        th = (np.arange(2 * m) + rng.uniform(-0.2, 0.2, 2 * m)) * (math.pi / m)
        rad = np.where(np.arange(2 * m) % 2 == 0, ro, 0.4 * ro)
        q = np.stack([cx + rad * np.cos(th), cy + rad * np.sin(th)], axis=1)
        out.append(np.clip(snap(q), 0.0, [width, height]))
    return out


def random_convex(rng, width, height, n, r_lo, r_hi, sides=(3, 8)):
    """n convex polygons of 3-8 vertices: sorted jittered angles on a circle
    of radius ~ U[r_lo, r_hi] centred inside the map; every other one listed
    clockwise."""
    out = []
    for k in range(n):
        m = int(rng.integers(sides[0], sides[1] + 1))
        r = rng.uniform(r_lo, r_hi)
        cx, cy = rng.uniform(r, width - r), rng.uniform(r, height - r)
        th = (np.arange(m) + rng.uniform(-0.3, 0.3, m)) * (2.0 * math.pi / m)
        q = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
        q = np.clip(snap(q), 0.0, [width, height])
        out.append(q[::-1].copy() if k % 2 else q)
    return out


def convex_map(seed, S=200.0, n_rects=6, n_convex=12):
    """Rectangles and convex polygons of 3-8 vertices in both orientations,
    start and target in opposite corners."""
    rng = np.random.default_rng(seed)
    s, t = snap([0.04 * S, 0.06 * S]), snap([0.96 * S, 0.94 * S])
    rects = random_rects(rng, S, S, n_rects, 0.04 * S, 0.15 * S, avoid=(s, t))
    polys = random_convex(rng, S, S, n_convex, 0.04 * S, 0.12 * S)
    return make_map(S, S, list(rects) + polys, s, t)


def nonconvex_map(seed, S=200.0, n_rects=6, n_stars=6):
    """Mixed obstacle set: rectangles and non-convex stars (a variant the
    polygon representation allows), start and target in opposite corners."""
    rng = np.random.default_rng(seed)
    s, t = snap([0.04 * S, 0.06 * S]), snap([0.96 * S, 0.94 * S])
    rects = random_rects(rng, S, S, n_rects, 0.04 * S, 0.15 * S, avoid=(s, t))
    stars = random_stars(rng, S, S, n_stars, 0.05 * S, 0.12 * S)
    return make_map(S, S, list(rects) + stars, s, t)


def make_map(width, height, polys, start, target, poly_vel=None, endpoint_vel=None):
    polys = [np.asarray(p, dtype=np.float64) for p in polys]
    ptr = np.zeros(len(polys) + 1, dtype=np.int32)
    for i, p in enumerate(polys):
        ptr[i + 1] = ptr[i] + len(p)
    verts = np.concatenate(polys, axis=0) if polys else np.zeros((0, 2))
    if poly_vel is None:
        poly_vel = np.zeros((len(polys), 2))
    if endpoint_vel is None:
        endpoint_vel = np.zeros(4)
    return MapSpec(float(width), float(height), ptr, snap(verts), snap(start), snap(target),
                   snap(poly_vel), snap(endpoint_vel))


def static_map(seed, S=100.0, n_rects=4, side=(5.0, 20.0), start=(5.0, 5.0),
               target=(95.0, 95.0)):
    """Single static plan: S x S map, n_rects axis-aligned rectangles with
    sides uniform in `side`, fixed start and target."""
    rng = np.random.default_rng(seed)
    s, t = np.array(start, float), np.array(target, float)
    rects = random_rects(rng, S, S, n_rects, *side, avoid=(s, t))
    return make_map(S, S, rects, s, t)


def random_static_maps(n, seed, S=100.0, n_rects=4, side=(5.0, 20.0), margin=1.0):
    """n static maps of the single-plan shape with random start and target
    (learned-initializer training and held-out sets), drawn vectorised:
    start/target uniform in [2, S-2]^2, rectangles as in static_map, any
    rectangle containing an endpoint (with margin) redrawn."""
    rng = np.random.default_rng(seed)
    st = snap(rng.uniform(2.0, S - 2.0, size=(n, 2, 2)))
    wh = snap(rng.uniform(*side, size=(n, n_rects, 2)))
    xy = snap(rng.uniform(0.0, 1.0, size=(n, n_rects, 2)) * (S - wh))
    for _ in range(1000):
        bad = np.zeros((n, n_rects), bool)
        for e in range(2):
            p = st[:, e, None, :]
            bad |= np.all((xy - margin <= p) & (p <= xy + wh + margin), axis=2)
        if not bad.any():
            break
        k = int(bad.sum())
        wh[bad] = snap(rng.uniform(*side, size=(k, 2)))
        xy[bad] = snap(rng.uniform(0.0, 1.0, size=(k, 2)) * (S - wh[bad]))
    maps = []
    for i in range(n):
        rects = [[[x, y], [x + w, y], [x + w, y + h], [x, y + h]]
                 for (x, y), (w, h) in zip(xy[i], wh[i])]
        maps.append(make_map(S, S, rects, st[i, 0], st[i, 1]))
    return maps


def learned_swarm(seed=0, instance=0, iters=50):
    """Planner shape the learned initializer serves: 8 groups x 32
    particles x 20 waypoints with the Table hyper8 rows, 1e3 per crossing,
    no truncation; proposals are perturbed by +-5% of the map."""
    hyper = HYPER8[np.arange(8)]
    return SwarmSpec(8, 32, 20, iters, hyper, alpha=1e3, beta=1, seed=seed, instance=instance,
                     pi_gamma=0.25, pi_radius=5.0)


def dynamic_map(seed, S=366.0, n_static=10, n_moving=20, side=(10.0, 40.0), vmax=2.0):
    """Paper-shaped dynamic scene: S x S map, static and moving rectangles
    (velocities uniform in +-vmax cells/frame per axis, bouncing off the
    walls), start near the left edge and target near the right edge, both
    moving vertically at 1 cell/frame."""
    rng = np.random.default_rng(seed)
    s = snap([0.05 * S, rng.uniform(0.25 * S, 0.75 * S)])
    t = snap([0.95 * S, rng.uniform(0.25 * S, 0.75 * S)])
    rects = random_rects(rng, S, S, n_static + n_moving, *side, avoid=(s, t), margin=2.0)
    vel = np.zeros((n_static + n_moving, 2))
    vel[n_static:] = snap(rng.uniform(-vmax, vmax, size=(n_moving, 2)))
    ev = np.array([0.0, rng.choice([-1.0, 1.0]), 0.0, rng.choice([-1.0, 1.0])])
    return make_map(S, S, rects, s, t, vel, ev)


def stress_map(seed, S=512.0, n_rects=500, n_quads=100):
    """Large-swarm stress scene: rectangles (sides 5-20) and convex quads
    (semi-axes 5-30) on an S x S map; start and target in opposite corners."""
    rng = np.random.default_rng(seed)
    s, t = snap([0.02 * S, 0.02 * S]), snap([0.98 * S, 0.98 * S])
    rects = random_rects(rng, S, S, n_rects, 5.0, 20.0, avoid=(s, t))
    quads = random_quads(rng, S, S, n_quads, 5.0, 30.0)
    return make_map(S, S, list(rects) + list(quads), s, t)


def batch_instance(i, seed_base=0):
    """Instance i of the ragged batch: W ~ U{8..32}, rectangles ~ U{4..100},
    particles per group ~ U{32..256} over 8 groups, map side ~ U{128..512};
    obstacle and endpoint motion as in dynamic_map, scaled to the map."""
    rng = np.random.default_rng([seed_base, i])
    S = float(rng.integers(128, 513))
    W = int(rng.integers(8, 33))
    n_rects = int(rng.integers(4, 101))
    N = int(rng.integers(32, 257))
    n_moving = (2 * n_rects) // 3
    lo, hi = 0.03 * S, 0.11 * S
    m = dynamic_map(int(rng.integers(1 << 31)), S=S, n_static=n_rects - n_moving,
                    n_moving=n_moving, side=(lo, hi))
    return m, dict(groups=8, particles=N, waypoints=W)


def flatten_hyper(rows):
    return f32(np.asarray(rows, dtype=np.float64).reshape(-1, 6))


def static_swarm(seed=0, groups=4, particles=32, waypoints=8, iters=50, variant="hyper1"):
    """Swarm of the single static plan.  variant 'hyper1': Table hyper1 in
    every group with the Tbest term off; 'hyper8': Table hyper8 rows."""
    if variant == "hyper1":
        hyper = np.tile(HYPER1_ROW, (groups, 1))
    else:
        hyper = HYPER8[np.arange(groups) % 8]
    return SwarmSpec(groups, particles, waypoints, iters, hyper, alpha=1e3, beta=1, seed=seed)


def dynamic_swarm(S, seed=0, groups=8, particles=170, waypoints=20, iters=50,
                  at_mode=2, hsef_every=10, use_pi=1, instance=0):
    """Swarm of the paper-shaped dynamic run: Table hyper8path start values,
    Table params_path penalty and PI fraction, truncation when the best
    improves by < 1e-3 (relative) over 5 iterations, online self-evolution
    every 10 iterations, PI radius 5% of the map."""
    pp = PARAMS_PATH
    return SwarmSpec(groups, particles, waypoints, iters, HYPER8PATH[np.arange(groups) % 8],
                     alpha=pp["alpha"], beta=pp["beta"], seed=seed, instance=instance,
                     use_pi=use_pi,
                     pi_gamma=pp["gamma"], pi_radius=0.05 * S, at_mode=at_mode, at_window=5,
                     at_delta=1e-3, hsef_every=hsef_every)
