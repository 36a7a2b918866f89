"""Seeded synthetic inputs: point clouds, transmitter/receiver layouts, materials.

This module only *generates inputs*. It holds none of the tracer's arithmetic
(no intersection, reflection, Fresnel or gain code), so that both the GPU
library and the CPU oracle can be fed the same arrays from it.

The paper's input is an augmented point cloud: per point a position, a surface
normal, a surface label and a material label (Sec. II, opening paragraph).
The paper's own scenes (a scanned corridor, Replica room 0) are not available,
so every scene here is a synthetic stand-in of the same kind: planar indoor
surfaces sampled on a cell-centred grid, optionally with position noise and
normal jitter as a scanner would produce.

Arrays are returned as numpy: pos float32[N,3], normal float32[N,3],
material uint16[N], surface uint32[N]; disk radius as a Python float.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Material values are proposals for synthetic tests, not measured data:
# (relative permittivity, conductivity S/m, scattering coefficient).
MATERIALS_BOX_ROOM = {
    "concrete": (5.0, 0.1, 0.0),
    "glass": (6.0, 0.05, 0.0),
    "wood": (2.0, 0.01, 0.0),
    "metal": (1.0, 1.0e7, 0.0),
}


@dataclass
class Scene:
    pos: np.ndarray
    normal: np.ndarray
    material: np.ndarray
    surface: np.ndarray
    radius: float
    n_labels: int
    n_surfaces: int
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def permuted(self, perm: np.ndarray) -> "Scene":
        """Same scene with points reordered: new point i is old point perm[i]."""
        return Scene(self.pos[perm].copy(), self.normal[perm].copy(),
                     self.material[perm].copy(), self.surface[perm].copy(),
                     self.radius, self.n_labels, self.n_surfaces, dict(self.info))


def _grid(extent_u: float, extent_v: float, h: float):
    """Cell-centred grid over [0,eu]x[0,ev] with spacing close to h (exact fit)."""
    nu = max(1, int(round(extent_u / h)))
    nv = max(1, int(round(extent_v / h)))
    hu, hv = extent_u / nu, extent_v / nv
    u = (np.arange(nu, dtype=np.float64) + 0.5) * hu
    v = (np.arange(nv, dtype=np.float64) + 0.5) * hv
    uu, vv = np.meshgrid(u, v, indexing="ij")
    return uu.ravel(), vv.ravel()


def _pack(pos, nrm, mat, surf, radius, n_labels, n_surfaces, info) -> Scene:
    return Scene(np.ascontiguousarray(pos, dtype=np.float32),
                 np.ascontiguousarray(nrm, dtype=np.float32),
                 np.ascontiguousarray(mat, dtype=np.uint16),
                 np.ascontiguousarray(surf, dtype=np.uint32),
                 float(radius), int(n_labels), int(n_surfaces), info)


# ---------------------------------------------------------------------------
# Empty box room (6 x 4 x 3 m) with a window and a door.
# ---------------------------------------------------------------------------
# Surface labels: 0 x=0 wall, 1 x=W wall, 2 y=0 wall, 3 y=D wall, 4 floor,
# 5 ceiling, 6 window (on x=W), 7 door (on y=0).
BOX_WINDOW = dict(face=1, u=(1.5, 3.0), v=(1.0, 2.0))   # (y, z) range on x=W
BOX_DOOR = dict(face=2, u=(1.5, 2.5), v=(0.0, 2.0))     # (x, z) range on y=0


def box_room(spacing: float = 0.05, radius: float = 0.03, size=(6.0, 4.0, 3.0),
             labels: str = "four", window: bool = True, door: bool = True) -> Scene:
    """Empty rectangular room sampled on every face, exact inward normals.

    labels="four": material labels concrete 0 (walls, ceiling), glass 1
    (window), wood 2 (floor), metal 3 (door).
    labels="surface": material label = surface label (8 labels), used where a
    per-surface material is to be learned.
    """
    W, D, H = size
    faces = [
        # (surface, fixed axis, fixed value, inward normal, (axis_u, ext_u), (axis_v, ext_v))
        (0, 0, 0.0, (1, 0, 0), (1, D), (2, H)),
        (1, 0, W, (-1, 0, 0), (1, D), (2, H)),
        (2, 1, 0.0, (0, 1, 0), (0, W), (2, H)),
        (3, 1, D, (0, -1, 0), (0, W), (2, H)),
        (4, 2, 0.0, (0, 0, 1), (0, W), (1, D)),
        (5, 2, H, (0, 0, -1), (0, W), (1, D)),
    ]
    P, Nn, S = [], [], []
    for sid, ax, val, nrm, (au, eu), (av, ev) in faces:
        u, v = _grid(eu, ev, spacing)
        p = np.zeros((u.size, 3))
        p[:, ax] = val
        p[:, au] = u
        p[:, av] = v
        s = np.full(u.size, sid, dtype=np.int64)
        if window and sid == BOX_WINDOW["face"]:
            m = ((u >= BOX_WINDOW["u"][0]) & (u <= BOX_WINDOW["u"][1])
                 & (v >= BOX_WINDOW["v"][0]) & (v <= BOX_WINDOW["v"][1]))
            s[m] = 6
        if door and sid == BOX_DOOR["face"]:
            m = ((u >= BOX_DOOR["u"][0]) & (u <= BOX_DOOR["u"][1])
                 & (v >= BOX_DOOR["v"][0]) & (v <= BOX_DOOR["v"][1]))
            s[m] = 7
        P.append(p)
        Nn.append(np.tile(np.asarray(nrm, dtype=np.float64), (u.size, 1)))
        S.append(s)
    pos = np.concatenate(P)
    nrm = np.concatenate(Nn)
    surf = np.concatenate(S)
    if labels == "four":
        mat = np.zeros_like(surf)
        mat[surf == 6] = 1
        mat[surf == 4] = 2
        mat[surf == 7] = 3
        n_labels = 4
    elif labels == "surface":
        mat = surf.copy()
        n_labels = 8
    else:
        raise ValueError(labels)
    info = dict(kind="box_room", size=size, spacing=spacing)
    return _pack(pos, nrm, mat, surf, radius, n_labels, 8, info)


def box_room_materials(labels: str = "four", scatter: float = 0.0) -> np.ndarray:
    """float64[n_labels, 3] (eps_r, sigma, S) for box_room()."""
    if labels == "four":
        rows = [MATERIALS_BOX_ROOM[k] for k in ("concrete", "glass", "wood", "metal")]
    else:
        c, g, w, m = (MATERIALS_BOX_ROOM[k] for k in ("concrete", "glass", "wood", "metal"))
        rows = [c, c, c, c, w, c, g, m]
    out = np.array(rows, dtype=np.float64)
    out[:, 2] = scatter
    return out


BOX_TX = (1.0, 1.0, 1.5)
BOX_RX = (5.0, 3.0, 1.2)


# ---------------------------------------------------------------------------
# Furnished office (12 x 8 x 3 m, 20 boxes, ~1M noisy points).
# ---------------------------------------------------------------------------
OFFICE_SIZE = (12.0, 8.0, 3.0)
OFFICE_TX = (6.0, 4.0, 2.5)
# (eps_r, sigma, S) for labels: walls, floor, ceiling, glass, metal door,
# three furniture materials. Proposals for synthetic tests.
OFFICE_MATERIALS = np.array([
    [5.0, 0.50, 0.3],
    [2.0, 0.10, 0.3],
    [2.9, 0.20, 0.3],
    [6.3, 0.30, 0.3],
    [1.0, 1.0e7, 0.3],
    [2.0, 0.10, 0.3],
    [2.6, 0.15, 0.3],
    [3.0, 0.05, 0.3],
], dtype=np.float64)


def office_rx() -> np.ndarray:
    """64 receivers on a 1.2 m-high grid: x = 0.75 + 1.5 i, y = 0.5 + 1.0 j."""
    xs = 0.75 + 1.5 * np.arange(8)
    ys = 0.5 + 1.0 * np.arange(8)
    xx, yy = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), np.full(64, 1.2)], 1).astype(np.float32)


def _box_distance(pt, c, half, yaw, height):
    """Euclidean distance from a point to a yawed box standing on the floor."""
    dx, dy = pt[0] - c[0], pt[1] - c[1]
    ca, sa = math.cos(yaw), math.sin(yaw)
    lx, ly = ca * dx + sa * dy, -sa * dx + ca * dy
    qx = max(abs(lx) - half[0], 0.0)
    qy = max(abs(ly) - half[1], 0.0)
    qz = max(pt[2] - height, 0.0, -pt[2])
    return math.sqrt(qx * qx + qy * qy + qz * qz)


def _office_boxes(rng, n_boxes, size, keep_clear, clearance=0.2):
    W, D, _ = size
    boxes = []
    tries = 0
    while len(boxes) < n_boxes:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place furniture")
        sx, sy = rng.uniform(0.4, 2.0, 2)
        hgt = rng.uniform(0.4, 2.0)
        yaw = rng.uniform(0.0, math.pi / 2)
        rad = 0.5 * math.hypot(sx, sy)
        cx = rng.uniform(0.1 + rad, W - 0.1 - rad)
        cy = rng.uniform(0.1 + rad, D - 0.1 - rad)
        half = (0.5 * sx, 0.5 * sy)
        if any(_box_distance(p, (cx, cy), half, yaw, hgt) < clearance for p in keep_clear):
            continue
        if any(math.hypot(cx - b["c"][0], cy - b["c"][1]) < rad + b["rad"] + 0.05 for b in boxes):
            continue
        boxes.append(dict(c=(cx, cy), half=half, yaw=yaw, h=hgt, rad=rad))
    return boxes


def _office_points(boxes, size, h):
    """Noise-free points, normals, surface labels for a given grid spacing."""
    W, D, H = size
    P, Nn, S = [], [], []
    faces = [
        (0, 0, 0.0, (1, 0, 0), (1, D), (2, H)),
        (1, 0, W, (-1, 0, 0), (1, D), (2, H)),
        (2, 1, 0.0, (0, 1, 0), (0, W), (2, H)),
        (3, 1, D, (0, -1, 0), (0, W), (2, H)),
        (4, 2, 0.0, (0, 0, 1), (0, W), (1, D)),
        (5, 2, H, (0, 0, -1), (0, W), (1, D)),
    ]
    for sid, ax, val, nrm, (au, eu), (av, ev) in faces:
        u, v = _grid(eu, ev, h)
        p = np.zeros((u.size, 3))
        p[:, ax] = val
        p[:, au] = u
        p[:, av] = v
        s = np.full(u.size, sid, dtype=np.int64)
        if sid == 1:  # window on the x=W wall
            s[(u >= 2.0) & (u <= 6.0) & (v >= 1.0) & (v <= 2.2)] = 6
        if sid == 2:  # door on the y=0 wall
            s[(u >= 2.0) & (u <= 3.0) & (v <= 2.1)] = 7
        P.append(p)
        Nn.append(np.tile(np.asarray(nrm, float), (u.size, 1)))
        S.append(s)
    sid = 8
    for b in boxes:
        ca, sa = math.cos(b["yaw"]), math.sin(b["yaw"])
        ex = np.array([ca, sa, 0.0])
        ey = np.array([-sa, ca, 0.0])
        c = np.array([b["c"][0], b["c"][1], 0.0])
        hx, hy, hz = b["half"][0], b["half"][1], b["h"]
        # four vertical sides and the top; outward normals
        sides = [(ex, ey, hx, hy), (-ex, -ey, hx, hy), (ey, -ex, hy, hx), (-ey, ex, hy, hx)]
        for nrm, tang, dn, dt in sides:
            u, v = _grid(2 * dt, hz, h)
            p = c + nrm * dn + np.outer(u - dt, tang) + np.outer(v, [0, 0, 1.0])
            P.append(p)
            Nn.append(np.tile(nrm, (u.size, 1)))
            S.append(np.full(u.size, sid, dtype=np.int64))
            sid += 1
        u, v = _grid(2 * hx, 2 * hy, h)
        p = c + np.outer(u - hx, ex) + np.outer(v - hy, ey) + np.array([0, 0, hz])
        P.append(p)
        Nn.append(np.tile([0, 0, 1.0], (u.size, 1)))
        S.append(np.full(u.size, sid, dtype=np.int64))
        sid += 1
    return np.concatenate(P), np.concatenate(Nn), np.concatenate(S), sid


def office(seed: int = 2507, target_points: int = 1_000_000, n_boxes: int = 20,
           pos_sigma: float = 0.005, normal_jitter_deg: float = 3.0,
           radius: float | None = None, size=OFFICE_SIZE) -> Scene:
    """Furnished office: 20 yawed boxes, grid tuned to ~target_points points.

    Positions get isotropic Gaussian noise (pos_sigma); normals get a Gaussian
    tangent-plane tilt with per-axis std tan(normal_jitter_deg).
    Material labels: walls 0, floor 1, ceiling 2, glass 3, door 4, furniture
    cycles 5/6/7 per box. Surface labels: 6 room faces, window 6, door 7, then
    5 faces per box.
    """
    rng = np.random.default_rng(seed)
    keep = [OFFICE_TX] + [tuple(r) for r in office_rx()]
    boxes = _office_boxes(rng, n_boxes, size, keep)
    # tune the spacing so that the point count is close to the target
    h = 0.02
    for _ in range(8):
        p, _, _, _ = _office_points(boxes, size, h)
        h *= math.sqrt(p.shape[0] / target_points)
    pos, nrm, surf, n_surf = _office_points(boxes, size, h)
    n = pos.shape[0]
    pos = pos + rng.normal(0.0, pos_sigma, size=(n, 3))
    if normal_jitter_deg > 0:
        # tangent basis per point
        a = np.where(np.abs(nrm[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        t1 = np.cross(nrm, a)
        t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
        t2 = np.cross(nrm, t1)
        s = math.tan(math.radians(normal_jitter_deg))
        g = rng.normal(0.0, s, size=(n, 2))
        nrm = nrm + g[:, :1] * t1 + g[:, 1:] * t2
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mat = np.zeros(n, dtype=np.int64)
    mat[surf == 4] = 1
    mat[surf == 5] = 2
    mat[surf == 6] = 3
    mat[surf == 7] = 4
    box_of = (surf - 8) // 5
    mat[surf >= 8] = 5 + (box_of[surf >= 8] % 3)
    r = h if radius is None else radius
    info = dict(kind="office", seed=seed, spacing=h, boxes=boxes, size=size)
    return _pack(pos, nrm, mat, surf, r, 8, n_surf, info)


def office_edges(sc: Scene):
    """Convex edges of the office furniture, for single-bounce diffraction:
    per box the four vertical edges and the four top edges (the edges on the
    floor and the room's corners are concave). Returns (rows float32[n, 12]:
    a xyz, b xyz, outward normal of face 0, of face n; labels int32[n, 2]:
    material of face 0 and face n)."""
    rows, labels = [], []
    for i, b in enumerate(sc.info["boxes"]):
        ca, sa = math.cos(b["yaw"]), math.sin(b["yaw"])
        ex, ey, ez = np.array([ca, sa, 0.0]), np.array([-sa, ca, 0.0]), np.array([0.0, 0.0, 1.0])
        c = np.array([b["c"][0], b["c"][1], 0.0])
        hx, hy, hz = b["half"][0], b["half"][1], b["h"]
        mat = 5 + i % 3
        for sx in (-1.0, 1.0):
            for sy in (-1.0, 1.0):
                p = c + sx * hx * ex + sy * hy * ey
                rows.append(np.concatenate([p, p + hz * ez, sx * ex, sy * ey]))
                labels.append((mat, mat))
        for nrm, tng, dn, dt in ((ex, ey, hx, hy), (-ex, ey, hx, hy), (ey, ex, hy, hx), (-ey, ex, hy, hx)):
            p = c + dn * nrm + hz * ez
            rows.append(np.concatenate([p - dt * tng, p + dt * tng, nrm, ez]))
            labels.append((mat, mat))
    return np.array(rows, np.float32), np.array(labels, np.int32)


# ---------------------------------------------------------------------------
# Small scenes for unit tests.
# ---------------------------------------------------------------------------
def random_disks(n: int, seed: int, extent: float = 2.0, radius: float = 0.15,
                 n_labels: int = 3, n_surfaces: int = 5) -> Scene:
    """Disks with uniform random centres in a cube and random normals."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-extent, extent, size=(n, 3))
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mat = rng.integers(0, n_labels, n)
    surf = rng.integers(0, n_surfaces, n)
    return _pack(pos, nrm, mat, surf, radius, n_labels, n_surfaces, dict(kind="random", seed=seed))


def plane_patch(x0, x1, y0, y1, spacing, radius, z=0.0, material=0, surface=0) -> Scene:
    """Horizontal grid of disks on z = const with normal +z."""
    u, v = _grid(x1 - x0, y1 - y0, spacing)
    pos = np.stack([u + x0, v + y0, np.full(u.size, z)], 1)
    nrm = np.tile([0.0, 0.0, 1.0], (u.size, 1))
    return _pack(pos, nrm, np.full(u.size, material), np.full(u.size, surface), radius,
                 material + 1, surface + 1, dict(kind="plane"))


def single_disk(center, normal, radius, material=0, surface=0) -> Scene:
    n = np.asarray(normal, float)
    n = n / np.linalg.norm(n)
    return _pack(np.asarray([center], float), n[None], [material], [surface], radius,
                 material + 1, surface + 1, dict(kind="disk"))


def noisy(sc: Scene, seed: int, pos_sigma: float = 0.005, normal_jitter_deg: float = 3.0,
          radius: float | None = None) -> Scene:
    """A copy with the office's scanner-like noise: isotropic Gaussian position
    noise and a Gaussian tangent-plane tilt of the normals."""
    rng = np.random.default_rng(seed)
    pos = sc.pos.astype(np.float64) + rng.normal(0.0, pos_sigma, size=sc.pos.shape)
    nrm = sc.normal.astype(np.float64)
    a = np.where(np.abs(nrm[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(nrm, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    g = rng.normal(0.0, math.tan(math.radians(normal_jitter_deg)), size=(sc.n, 2))
    nrm = nrm + g[:, :1] * t1 + g[:, 1:] * t2
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    info = dict(sc.info, noise=(seed, pos_sigma, normal_jitter_deg))
    return _pack(pos, nrm, sc.material, sc.surface, sc.radius if radius is None else radius, sc.n_labels,
                 sc.n_surfaces, info)


def concat(scenes) -> Scene:
    pos = np.concatenate([s.pos for s in scenes])
    nrm = np.concatenate([s.normal for s in scenes])
    mat = np.concatenate([s.material for s in scenes])
    surf = np.concatenate([s.surface for s in scenes])
    radius = scenes[0].radius
    return _pack(pos, nrm, mat, surf, radius, int(mat.max()) + 1, int(surf.max()) + 1,
                 dict(kind="concat"))


# ---------------------------------------------------------------------------
# Robot trajectory (batched transmitter poses) and hidden materials.
# ---------------------------------------------------------------------------
def trajectory(seed: int = 4021, n: int = 256, z: float = 0.5, step: float = 0.1,
               turn_deg: float = 15.0, lo=(0.5, 0.5), hi=(5.5, 3.5),
               min_rays: int = 1 << 16, max_rays: int = 1 << 20):
    """Random-walk transmitter poses and per-pose ray counts.

    Returns (tx float32[n,3], n_rays int64[n]).
    """
    rng = np.random.default_rng(seed)
    x, y, hd = 1.0, 1.0, 0.0
    tx = np.zeros((n, 3))
    for i in range(n):
        tx[i] = (x, y, z)
        hd += math.radians(rng.normal(0.0, turn_deg))
        x = min(max(x + step * math.cos(hd), lo[0]), hi[0])
        y = min(max(y + step * math.sin(hd), lo[1]), hi[1])
    rays = rng.integers(min_rays, max_rays + 1, n)
    return tx.astype(np.float32), rays.astype(np.int64)


def hidden_materials(seed: int = 7, n_labels: int = 8, scatter=None) -> np.ndarray:
    """float64[n_labels, 3]: eps_r ~ U[2,10], sigma ~ log-U[1e-3, 1], S = 0 or ~ U[scatter]."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(2.0, 10.0, n_labels)
    sig = np.exp(rng.uniform(math.log(1e-3), math.log(1.0), n_labels))
    S = np.zeros(n_labels) if scatter is None else rng.uniform(scatter[0], scatter[1], n_labels)
    return np.stack([eps, sig, S], 1)


def random_links(seed: int, n_sets: int, n_rx: int, lo=(0.3, 0.3, 0.3), hi=(5.7, 3.7, 2.7)):
    """Random TX and RX positions inside the box room: (tx[n_sets,3], rx[n_sets,n_rx,3])."""
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo), np.asarray(hi)
    tx = rng.uniform(lo, hi, size=(n_sets, 3))
    rx = rng.uniform(lo, hi, size=(n_sets, n_rx, 3))
    return tx.astype(np.float32), rx.astype(np.float32)


def stratified_ray_ids(n_rays: int, n_sample: int) -> np.ndarray:
    """Evenly spread ray indices j = floor((i + 1/2) N / n) used for sampled parity."""
    i = np.arange(n_sample, dtype=np.float64)
    return np.floor((i + 0.5) * n_rays / n_sample).astype(np.int64)
