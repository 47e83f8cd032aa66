"""Seeded synthetic particle sets shaped like the paper's scenes.

This module only draws inputs: site positions, prescribed volumes, initial
weights and velocities. It holds none of the method's arithmetic, so both the
FP64 oracle (test infrastructure) and the HIP path can be fed from it.

Canonical form of every scene:
  * positions are drawn in float64 and rounded to float32 (the float32 values
    ARE the input; the oracle promotes them back to float64 exactly);
  * prescribed volumes ``nu`` and weights ``psi`` are float64;
  * the domain is the unit box [0,1]^3.

Scene recipes (sizes follow the workloads the solver is measured on):
  slab_uniform   N sites uniform in [0,1]^2 x [0,0.4], nu = 0.3/N       (1,000 sites)
  dam_break      jittered cubic lattice filling the lower 40% of the box,
                 nu summing to 0.35                                       (100,000 sites)
  splash         lattice slab (60%) + 200 log-normal spheres (40%),
                 log-normal nu summing to 0.3, random velocities          (2,000,000 sites)
  batch          256 instances with N log-uniform in [500, 50,000]
  The default start weight gives every ball the radius 1.2 (3 nu / 4 pi)^(1/3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BOX_LO = (0.0, 0.0, 0.0)
BOX_HI = (1.0, 1.0, 1.0)


@dataclass
class Scene:
    name: str
    x: np.ndarray          # float32 [N]
    y: np.ndarray          # float32 [N]
    z: np.ndarray          # float32 [N]
    nu: np.ndarray         # float64 [N]  prescribed volumes
    psi0: np.ndarray       # float64 [N]  start weights (psi = r^2)
    vel: np.ndarray | None = None   # float64 [N,3] (splash only)
    box: tuple = (BOX_LO, BOX_HI)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def xyz64(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1).astype(np.float64)


def default_psi0(nu: np.ndarray, radius_factor: float = 1.2) -> np.ndarray:
    """Start weights: ball radius radius_factor * (3 nu / 4 pi)^(1/3), psi = r^2."""
    r = radius_factor * np.cbrt(3.0 * np.asarray(nu, np.float64) / (4.0 * math.pi))
    return r * r


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _jittered_lattice(rng, h, nx, ny, nz, origin=(0.0, 0.0, 0.0), jitter=0.3):
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    p = np.stack([(i.ravel() + 0.5) * h + origin[0],
                  (j.ravel() + 0.5) * h + origin[1],
                  (k.ravel() + 0.5) * h + origin[2]], axis=1)
    p += rng.uniform(-jitter * h, jitter * h, size=p.shape)
    return p


def _keep_lowest_z(p, n):
    order = np.lexsort((np.arange(p.shape[0]), p[:, 2]))  # z, ties by index
    return p[np.sort(order[:n])]


def _inside_box(p, eps=1e-6):
    return np.clip(p, eps, 1.0 - eps)


def slab_uniform(n: int = 1000, seed: int = 0, zmax: float = 0.4, total: float = 0.3) -> Scene:
    """N sites uniform in [0,1]^2 x [0,zmax], equal volumes summing to ``total``."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, size=(n, 3))
    p[:, 2] *= zmax
    p = _inside_box(p)
    nu = np.full(n, total / n)
    return Scene("slab_uniform", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, default_psi0(nu),
                 meta={"seed": seed, "n": n})


def dam_break(n: int = 100_000, seed: int = 0, fill: float = 0.4, total: float = 0.35,
              jitter: float = 0.3) -> Scene:
    """Jittered cubic lattice (jitter +-0.3 spacing) filling the lower ``fill`` of the box."""
    rng = np.random.default_rng(seed)
    h = (fill / n) ** (1.0 / 3.0)
    # columns at (i + 1/2) h while the jittered lattice stays inside the box:
    # (nxy - 1/2) h + jitter h < 1 (63 columns at 100,000 sites)
    nxy = int(math.floor(1.0 / h + 0.5 - jitter - 1e-9))
    nz = int(math.ceil(n / (nxy * nxy))) + 1
    p = _jittered_lattice(rng, h, nxy, nxy, nz, jitter=jitter)
    p = _keep_lowest_z(p, n)
    p = _inside_box(p)
    nu = np.full(n, total / n)
    return Scene("dam_break", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, default_psi0(nu),
                 meta={"seed": seed, "n": n, "h": h, "lattice": (nxy, nxy, nz)})


def _sphere_points(rng, centre, R, count, jitter=0.3):
    """``count`` points of a jittered lattice closest to ``centre`` (spacing fit to the ball)."""
    if count <= 0:
        return np.zeros((0, 3))
    vol = 4.0 / 3.0 * math.pi * R ** 3
    s = (vol / count) ** (1.0 / 3.0)
    for _ in range(200):
        m = int(math.ceil(R / s)) + 2
        ax = (np.arange(-m, m + 1) + 0.0) * s
        gx, gy, gz = np.meshgrid(ax, ax, ax, indexing="ij")
        q = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        q += rng.uniform(-jitter * s, jitter * s, size=q.shape)
        d2 = (q * q).sum(1)
        inside = d2 <= R * R
        if inside.sum() >= count:
            order = np.argsort(d2, kind="stable")[:count]
            return q[order] + np.asarray(centre)
        s *= 0.99
    raise RuntimeError("sphere lattice could not be filled")


def splash(n: int = 2_000_000, seed: int = 0, n_spheres: int = 200, slab_frac: float = 0.6,
           total: float = 0.3) -> Scene:
    """Crown-splash-like scene: lattice slab + log-normal spheres, log-normal volumes."""
    rng = np.random.default_rng(seed)
    n_slab = int(round(slab_frac * n))
    n_sph = n - n_slab
    h = (0.2 / n_slab) ** (1.0 / 3.0)
    nxy = int(math.floor(1.0 / h))
    nz = int(math.ceil(n_slab / (nxy * nxy))) + 1
    slab = _keep_lowest_z(_jittered_lattice(rng, h, nxy, nxy, nz), n_slab)
    radii = np.clip(rng.lognormal(math.log(0.03), 0.5, size=n_spheres), 0.01, 0.12)
    centres = []
    for R in radii:
        for _ in range(100000):
            c = np.array([rng.uniform(R, 1 - R), rng.uniform(R, 1 - R), rng.uniform(0.2 + R, 1 - R)])
            if all(np.linalg.norm(c - c2) > R + R2 for c2, R2 in centres):
                centres.append((c, R))
                break
        else:
            raise RuntimeError("could not place sphere")
    vols = np.array([R ** 3 for _, R in centres])
    quota = vols / vols.sum() * n_sph
    counts = np.floor(quota).astype(np.int64)
    rem = n_sph - counts.sum()
    counts[np.argsort(-(quota - counts), kind="stable")[:rem]] += 1
    parts = [slab] + [_sphere_points(rng, c, R, int(k)) for (c, R), k in zip(centres, counts)]
    p = _inside_box(np.concatenate(parts, axis=0))
    nu = rng.lognormal(0.0, 0.2, size=n)
    nu *= total / nu.sum()
    vel = rng.normal(0.0, 0.5, size=(n, 3))
    # start weights: one common weight (a Voronoi start). Per-site radii from the
    # log-normal nu leave light sites swallowed by heavy neighbours in the crowded
    # spheres (empty or near-empty start cells, so a KMT floor near zero).
    psi0 = np.full(n, default_psi0(np.array([nu.mean()]))[0])
    return Scene("splash", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, psi0, vel=vel,
                 meta={"seed": seed, "n": n, "n_slab": n_slab, "spheres": len(centres)})


def sphere_cluster(n: int, seed: int, total: float = 0.35, fill: float = 0.40) -> Scene:
    """K in 2..6 overlapping spheres of a common radius; the lattice fills their union."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 7))
    centres = rng.uniform(0.25, 0.75, size=(k, 3))
    s = (fill / n) ** (1.0 / 3.0)
    m = int(math.floor(1.0 / s))
    lat = _jittered_lattice(rng, s, m, m, m)
    d2 = ((lat[:, None, :] - centres[None, :, :]) ** 2).sum(-1).min(1)
    lo, hi = 0.0, 1.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if (d2 <= mid * mid).sum() >= n:
            hi = mid
        else:
            lo = mid
    order = np.argsort(d2, kind="stable")[:n]
    p = _inside_box(lat[np.sort(order)])
    nu = np.full(n, total / n)
    return Scene("sphere_cluster", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, default_psi0(nu),
                 meta={"seed": seed, "n": n, "spheres": k, "R": hi})


def overpacked_sphere(n: int = 2500, over: float = 1.72, seed: int = 0, R: float = 0.15) -> Scene:
    """One sphere of radius R at the box centre filled with a jittered lattice of n
    sites whose prescribed volumes add up to `over` times the sphere's volume (the
    packing of the splash scene's spheres): the converged balls overlap hundreds of
    neighbours."""
    rng = np.random.default_rng(seed)
    vol = 4.0 / 3.0 * math.pi * R ** 3
    h = (vol / n) ** (1.0 / 3.0)
    g = np.arange(-R - h, R + h, h)
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = p + rng.uniform(-0.3 * h, 0.3 * h, p.shape)
    p = p[np.argsort(np.linalg.norm(p, axis=1), kind="stable")[:n]] + 0.5
    nu = np.full(n, over * vol / n)
    return Scene("overpacked_sphere", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, default_psi0(nu),
                 meta={"seed": seed, "n": n, "over": over, "h": h})


def batch_instances(count: int = 256, base_seed: int = 1000, n_lo: int = 500, n_hi: int = 50_000):
    """Independent instances of uneven size: slab layout for even seeds, sphere cluster for odd."""
    out = []
    for b in range(count):
        seed = base_seed + b
        rng = np.random.default_rng(seed)
        nb = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        if seed % 2 == 0:
            sc = dam_break(nb, seed=seed)
        else:
            sc = sphere_cluster(nb, seed=seed)
        sc.meta["instance"] = b
        out.append(sc)
    return out


def advect(scene: Scene, dt: float = 2e-3) -> Scene:
    """x <- x + dt v with mirror reflection at the walls (velocity component negated)."""
    assert scene.vel is not None
    p = scene.xyz64() + dt * scene.vel
    v = scene.vel.copy()
    lo = p < 0.0
    p[lo] = -p[lo]
    v[lo] = -v[lo]
    hi = p > 1.0
    p[hi] = 2.0 - p[hi]
    v[hi] = -v[hi]
    p = _inside_box(p)
    return Scene(scene.name, _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), scene.nu.copy(),
                 scene.psi0.copy(), vel=v, box=scene.box, meta=dict(scene.meta))


def with_velocity(scene: Scene, seed: int, sigma: float = 0.5) -> Scene:
    rng = np.random.default_rng(seed)
    scene.vel = rng.normal(0.0, sigma, size=(scene.n, 3))
    return scene


def random_small(n: int, seed: int, lo: float = 0.15, hi: float = 0.85, r_lo: float = 0.08,
                 r_hi: float = 0.22) -> Scene:
    """Tiny random configurations for brute-force pins (overlapping balls, walls nearby)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(lo, hi, size=(n, 3))
    r = rng.uniform(r_lo, r_hi, size=n)
    nu = np.full(n, 1e-3)
    return Scene("random_small", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, r * r,
                 meta={"seed": seed, "n": n})


CONFIGS = {
    "c1_slab_1k": lambda seed=0: slab_uniform(1000, seed),
    "c2_dam_100k": lambda seed=0: dam_break(100_000, seed),
    "c3_splash_2m": lambda seed=0: splash(2_000_000, seed),
}


# An L-shaped prism, the unit box without the quarter x > 1/2, y > 1/2: a non-convex
# polyhedral domain given as convex pieces (each a list of planes (n, c), n.x <= c, with
# the wall each plane bounds, or -1 for a plane between two pieces). Walls: 0 x = 0,
# 1 y = 0, 2 z = 0, 3 z = 1, 4 x = 1, 5 y = 1, 6 x = 1/2 (for y > 1/2), 7 y = 1/2 (for
# x > 1/2). Every plane of a piece lies wholly on a wall or wholly between two pieces.
L_WALLS = 8
L_VOLUME = 0.75
L_WALL_AREAS = (1.0, 1.0, 0.75, 0.75, 0.5, 0.5, 0.5, 0.5)


def _slab_planes(x0, x1, y0, y1, z0, z1, ids):
    """The six planes of the box [x0,x1] x [y0,y1] x [z0,z1] (-x, +x, -y, +y, -z, +z) and
    their wall ids."""
    planes = [[-1.0, 0.0, 0.0, -x0], [1.0, 0.0, 0.0, x1], [0.0, -1.0, 0.0, -y0], [0.0, 1.0, 0.0, y1],
              [0.0, 0.0, -1.0, -z0], [0.0, 0.0, 1.0, z1]]
    return np.array(planes), np.array(ids, np.int32)


def l_shape_pieces(split_z: bool = False):
    """The L-shaped prism as 3 convex pieces (2 x 2 x 1 quarters less one), or 6 with each
    also cut at z = 1/2. Returns the list of (planes [6, 4], wall ids [6])."""
    quarters = [((0.0, 0.5), (0.0, 0.5), (0, -1, 1, -1)),
                ((0.5, 1.0), (0.0, 0.5), (-1, 4, 1, 7)),
                ((0.0, 0.5), (0.5, 1.0), (0, 6, -1, 5))]
    zs = [((0.0, 0.5), (2, -1)), ((0.5, 1.0), (-1, 3))] if split_z else [((0.0, 1.0), (2, 3))]
    pieces = []
    for (x0, x1), (y0, y1), wxy in quarters:
        for (z0, z1), wz in zs:
            pieces.append(_slab_planes(x0, x1, y0, y1, z0, z1, list(wxy) + list(wz)))
    return pieces


def in_l_shape(p: np.ndarray, eps: float = 1e-6) -> np.ndarray:
    """Points strictly inside the L-shaped prism (by eps)."""
    inside_box = np.all((p > eps) & (p < 1.0 - eps), axis=1)
    cut = (p[:, 0] > 0.5 - eps) & (p[:, 1] > 0.5 - eps)
    return inside_box & ~cut


def l_shape_sites(n: int, seed: int, spread: float = 0.15) -> Scene:
    """n sites uniform in the L-shaped prism, nu = 0.5 |L| / n, start radii the default
    start's times a log-normal factor (sigma `spread`). The sites keep 1e-4 off the planes
    x, y, z = 1/2 between the pieces of l_shape_pieces (a site must not lie on one)."""
    rng = np.random.default_rng(seed)
    pts = []
    while sum(len(q) for q in pts) < n:
        q = rng.uniform(0.0, 1.0, (2 * n, 3))
        off = np.all(np.abs(q - 0.5) > 1e-4, axis=1)
        pts.append(q[in_l_shape(q, 1e-4) & off])
    p = np.concatenate(pts)[:n]
    nu = np.full(n, 0.5 * L_VOLUME / n)
    psi = default_psi0(nu) * np.exp(2.0 * spread * rng.standard_normal(n))
    return Scene(f"l_shape_{n}", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, psi)


def l_shape_crowded(n: int = 2500, seed: int = 0, over: float = 1.72, R: float = 0.15,
                    radius_factor: float = 3.0) -> Scene:
    """The over-packed sphere (jittered lattice, volumes `over` times the sphere's) centred
    at (0.36, 0.36, 0.5) in the L-shaped prism, next to the planes between its pieces and
    the re-entrant edge; the few sites outside the prism are dropped. The start radii are
    radius_factor (3 nu / 4 pi)^(1/3): equal weights (the Voronoi cells) with balls that
    reach hundreds of neighbours, so that the cells are crowded."""
    sc = overpacked_sphere(n, over, seed, R)
    p = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64) + np.array([-0.14, -0.14, 0.0])
    keep = in_l_shape(p, 1e-4)
    p = p[keep]
    nu = sc.nu[keep]
    return Scene("l_shape_crowded", _f32(p[:, 0]), _f32(p[:, 1]), _f32(p[:, 2]), nu, default_psi0(nu, radius_factor))
