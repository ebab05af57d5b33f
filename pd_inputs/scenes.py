"""Seeded scene descriptions: mesh, Dirichlet set, collision-prone region,
collision proxies, material constant and obstacle motion.

Everything here is an *input* to the method.  The obstacle schedules only say
where the spheres are at each step; testing proxies against them is part of
the method and lives in the oracle and in the GPU kernels separately.
"""
from dataclasses import dataclass, field
from typing import Callable, Optional
import numpy as np

from .grid import kuhn_grid, layer_mask

YOUNG_E = 1.0e5
POISSON_NU = 0.45


def lame_mu(E=YOUNG_E, nu=POISSON_NU):
    """Shear modulus mu = E / (2 (1 + nu)); lambda is not used by the method."""
    return E / (2.0 * (1.0 + nu))


@dataclass
class SphereSchedule:
    """Rigid spheres pushed into the top face.

    centers(step) -> (3, ns) float64, radii -> (ns,) float64.
    """
    base_xy: np.ndarray            # (2, ns)
    radii: np.ndarray              # (ns,)
    top_z: float
    depth_rate: np.ndarray         # (ns,) penetration depth per step
    drift: Optional[np.ndarray] = None   # (2, ns) lateral drift per step

    def centers(self, step):
        xy = self.base_xy.copy()
        if self.drift is not None:
            xy = xy + self.drift * step
        z = self.top_z + self.radii - self.depth_rate * step
        return np.vstack([xy, z[None, :]]).astype(np.float64)


@dataclass
class Scene:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    mu: float
    rest: np.ndarray               # (3, n) float64
    tets: np.ndarray               # (4, T) int32
    dirichlet: np.ndarray          # (n,) bool
    region: np.ndarray             # (n,) bool  collision-prone nodes x2
    proxies: np.ndarray            # (np,) int64 global ids of proxy nodes (conforming)
    k_pen: float
    spheres: Optional[SphereSchedule] = None
    outer_iters: int = 10
    inner_iters: int = 1
    steps: int = 10
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.rest.shape[1]

    @property
    def n_tets(self):
        return self.tets.shape[1]

    def region_ids(self):
        """Region nodes that are unknowns, ascending global id (region-local order)."""
        return np.nonzero(self.region & ~self.dirichlet)[0]

    def proxy_local(self):
        """Proxy positions in region-local numbering."""
        rid = self.region_ids()
        pos = np.full(self.n_nodes, -1, dtype=np.int64)
        pos[rid] = np.arange(rid.size)
        loc = pos[self.proxies]
        assert (loc >= 0).all()
        return loc.astype(np.int32)


def _grid_scene(name, nx, ny, nz, h, region_layers, seed, k_pen, **kw):
    rest, tets = kuhn_grid(nx, ny, nz, h)
    dirichlet = layer_mask(nx, ny, nz, [0])
    region = layer_mask(nx, ny, nz, region_layers)
    proxies = np.nonzero(layer_mask(nx, ny, nz, [nz]))[0].astype(np.int64)
    return Scene(name=name, nx=nx, ny=ny, nz=nz, h=h, mu=lame_mu(), rest=rest, tets=tets,
                 dirichlet=dirichlet, region=region, proxies=proxies, k_pen=k_pen,
                 seed=seed, **kw)


def scene_cube8(seed=1):
    """8x8x8 unit cube (h = 1/8), bottom pinned, region = top face (81 nodes),
    one sphere of radius 0.3 pushed 0.01 per step into the top face at a
    seeded lateral offset; k = 1e6; 10 steps of 10 PD iterations."""
    nx = ny = nz = 8
    h = 1.0 / 8
    rng = np.random.default_rng(seed)
    off = rng.uniform(-h, h, size=2)
    sph = SphereSchedule(base_xy=np.array([[0.5 + off[0]], [0.5 + off[1]]]),
                         radii=np.array([0.3]), top_z=1.0, depth_rate=np.array([0.01]))
    return _grid_scene("cube8", nx, ny, nz, h, [nz], seed, 1.0e6, spheres=sph,
                       outer_iters=10, inner_iters=1, steps=10)


def scene_slab56(seed=2, drift=False):
    """56x56x32 cells (h = 1), bottom pinned, region = top two node layers
    (6,498 nodes), proxies = top face; 16 seeded spheres (centres U[2,54]^2,
    radius U[0.5,2]) pressed in at depth_i(s) = d_i r_i s / 100 with
    d_i ~ U[0.2,0.8]; k = 1e6; 100 steps of 10 PD iterations.
    With drift=True every sphere also moves laterally U[-0.25,0.25]^2 per step."""
    nx, ny, nz = 56, 56, 32
    rng = np.random.default_rng(seed)
    ns = 16
    xy = rng.uniform(2.0, 54.0, size=(2, ns))
    r = rng.uniform(0.5, 2.0, size=ns)
    d = rng.uniform(0.2, 0.8, size=ns)
    dr = rng.uniform(-0.25, 0.25, size=(2, ns)) if drift else None
    sph = SphereSchedule(base_xy=xy, radii=r, top_z=float(nz), depth_rate=d * r / 100.0,
                         drift=dr)
    return _grid_scene("slab56", nx, ny, nz, 1.0, [nz - 1, nz], seed, 1.0e6, spheres=sph,
                       outer_iters=10, inner_iters=1, steps=100)


def slab56_trajectory(seed):
    """Sphere trajectory on the 56 x 56 x 32 slab for the learned warm start:
    16 spheres (centres U[8,48]^2, radius U[0.5,2]) pressed in at
    depth_i(s) = d_i r_i s / 40 with d_i ~ U[0.2,0.8], each drifting
    laterally U[-0.2,0.2]^2 per frame; frames s = 1, 2, ... ."""
    rng = np.random.default_rng(seed)
    ns = 16
    xy = rng.uniform(8.0, 48.0, size=(2, ns))
    r = rng.uniform(0.5, 2.0, size=ns)
    d = rng.uniform(0.2, 0.8, size=ns)
    dr = rng.uniform(-0.2, 0.2, size=(2, ns))
    return SphereSchedule(base_xy=xy, radii=r, top_z=32.0, depth_rate=d * r / 40.0, drift=dr)


def scene_small(nx, ny, nz, h=1.0, region_top_layers=2, seed=7, n_spheres=2,
                depth_frac=0.02, k_pen=1.0e6):
    """Small grids for exhaustive checks: region = the top `region_top_layers`
    node layers, proxies = top face, a few seeded spheres."""
    rng = np.random.default_rng(seed)
    layers = list(range(nz + 1 - region_top_layers, nz + 1))
    xy = np.vstack([rng.uniform(0.2 * nx * h, 0.8 * nx * h, n_spheres),
                    rng.uniform(0.2 * ny * h, 0.8 * ny * h, n_spheres)])
    r = rng.uniform(0.6, 1.5, n_spheres) * h
    sph = SphereSchedule(base_xy=xy, radii=r, top_z=nz * h,
                         depth_rate=np.full(n_spheres, depth_frac * h * 5))
    return _grid_scene(f"small{nx}x{ny}x{nz}", nx, ny, nz, h, layers, seed, k_pen,
                       spheres=sph, outer_iters=3, inner_iters=1, steps=3)


def scene_irregular(nx=12, ny=10, nz=9, h=1.0, jitter=0.1, region_radius=None, seed=9,
                    k_pen=1.0e6):
    """Irregular stand-in for an anatomical mesh: a Kuhn grid whose node
    positions are jittered by U[-jitter, jitter] h per coordinate (seeded),
    bottom layer pinned, and a collision-prone region shaped as a cap, the
    nodes within region_radius (default 0.35 min(nx, ny) h) of a seeded point
    of the top face, so the breadth-first levels of the interior from the
    region have uneven widths.  Proxies = top-face nodes of the region; one
    sphere above the cap centre."""
    rng = np.random.default_rng(seed)
    rest, tets = kuhn_grid(nx, ny, nz, h)
    rest = rest + rng.uniform(-jitter, jitter, size=rest.shape) * h
    dirichlet = layer_mask(nx, ny, nz, [0])
    if region_radius is None:
        region_radius = 0.35 * min(nx, ny) * h
    c = np.array([rng.uniform(0.3, 0.7) * nx * h, rng.uniform(0.3, 0.7) * ny * h, nz * h])
    region = np.linalg.norm(rest - c[:, None], axis=0) <= region_radius
    top = layer_mask(nx, ny, nz, [nz])
    proxies = np.nonzero(top & region)[0].astype(np.int64)
    sph = SphereSchedule(base_xy=c[:2, None].copy(), radii=np.array([0.3 * region_radius]),
                         top_z=nz * h, depth_rate=np.array([0.05 * h]))
    return Scene(name=f"irregular{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, mu=lame_mu(),
                 rest=rest, tets=tets, dirichlet=dirichlet, region=region, proxies=proxies,
                 k_pen=k_pen, spheres=sph, outer_iters=3, inner_iters=1, steps=3, seed=seed)


def random_penalty_set(rng, n_proxy, m_region, lo=0.01, hi=0.05):
    """Solver-benchmark penalty set: a random subset of proxies (between lo*m
    and hi*m of them) with target offsets drawn U[0, 0.5] downward along z.
    Returns (proxy positions, depth offsets)."""
    cnt = int(rng.integers(int(np.ceil(lo * m_region)), int(np.floor(hi * m_region)) + 1))
    cnt = min(cnt, n_proxy)
    sel = np.sort(rng.choice(n_proxy, size=cnt, replace=False))
    depth = rng.uniform(0.0, 0.5, size=cnt)
    return sel, depth


@dataclass
class JawSchedule:
    """Prescribed rotation of the bottom face about an x-parallel hinge at
    (y = hinge_y, z = 0): the front starts open by theta0 (front moved down),
    then closes at rate per step, while a roll about the z axis grows to
    roll_max so that contact starts at one corner.  Positive angles move the
    front (y < hinge_y) up."""
    hinge_y: float
    theta0: float          # radians, opening at step 0
    rate: float            # radians per step (closing)
    roll_max: float        # radians
    steps: int

    def angles(self, step):
        th = -self.theta0 + self.rate * step
        ps = self.roll_max * min(step, self.steps) / max(self.steps, 1)
        return th, ps

    def positions(self, rest_pts, step):
        """Prescribed positions (3, k) of the given rest points."""
        th, ps = self.angles(step)
        c, s = np.cos(th), np.sin(th)
        rel = rest_pts - np.array([[0.0], [self.hinge_y], [0.0]])
        y = c * rel[1] + s * rel[2]
        z = -s * rel[1] + c * rel[2]
        out = np.vstack([rel[0], y, z]) + np.array([[0.0], [self.hinge_y], [0.0]])
        cx = 0.5 * (rest_pts[0].min() + rest_pts[0].max())
        cr, sr = np.cos(ps), np.sin(ps)
        x0 = out[0] - cx
        y0 = out[1] - self.hinge_y
        out[0] = cx + cr * x0 - sr * y0
        out[1] = self.hinge_y + sr * x0 + cr * y0
        return out


@dataclass
class SlitScene:
    name: str
    rest: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    region: np.ndarray
    pairs: np.ndarray          # (2, P) global ids (lower lip, upper lip)
    bottom: np.ndarray         # global ids of the prescribed bottom face
    jaw: JawSchedule
    k_pen: float
    mu: float
    h: float
    meta_nx: int = 0
    meta_zs: int = 0
    meta_ys_end: int = 0

    @property
    def n_nodes(self):
        return self.rest.shape[1]

    @property
    def n_tets(self):
        return self.tets.shape[1]

    def region_ids(self):
        return np.nonzero(self.region & ~self.dirichlet)[0]

    def pairs_local(self):
        rid = self.region_ids()
        pos = np.full(self.n_nodes, -1, dtype=np.int64)
        pos[rid] = np.arange(rid.size)
        loc = pos[self.pairs]
        assert (loc >= 0).all()
        return loc.astype(np.int32)

    def prescribed(self, x, step):
        """x with the bottom face moved to the jaw pose of `step` (top stays at rest)."""
        x = x.copy()
        x[:, self.bottom] = self.jaw.positions(self.rest[:, self.bottom], step)
        return x


def scene_slit(nx=64, ny=64, nz=40, zs=20, ys_end=46, h=1.0, seed=5, steps=10,
               k_pen=5.0e5):
    """Self-contact stress case: a zero-thickness slit on k = zs over
    j < ys_end (two lips), top face fixed, bottom face rotated about the back
    hinge (jaw).  Region = node layers zs-1, zs (both lips) and zs+1 within the
    slit footprint (j <= ys_end); collision pairs = the lip twins."""
    from .grid import kuhn_grid_slit, grid_node_id
    rest, tets, twins = kuhn_grid_slit(nx, ny, nz, h, zs, ys_end)
    n0 = (nx + 1) * (ny + 1) * (nz + 1)
    n = rest.shape[1]
    kk = np.zeros(n, dtype=np.int64)
    jj = np.zeros(n, dtype=np.int64)
    kk[:n0] = np.arange(n0) // ((nx + 1) * (ny + 1))
    jj[:n0] = (np.arange(n0) // (nx + 1)) % (ny + 1)
    kk[n0:] = zs
    jj[n0:] = (twins[0] // (nx + 1)) % (ny + 1)
    top = kk == nz
    bottom = np.nonzero(kk == 0)[0]
    dirichlet = top | (kk == 0)
    region = np.isin(kk, [zs - 1, zs, zs + 1]) & (jj <= ys_end)
    rng = np.random.default_rng(seed)
    jaw = JawSchedule(hinge_y=ny * h, theta0=np.deg2rad(2.0),
                      rate=np.deg2rad(rng.uniform(0.4, 0.8)),
                      roll_max=np.deg2rad(rng.uniform(0.5, 1.5)), steps=steps)
    return SlitScene(name=f"slit{nx}x{ny}x{nz}", rest=rest, tets=tets, dirichlet=dirichlet,
                     region=region, pairs=twins, bottom=bottom, jaw=jaw, k_pen=k_pen,
                     mu=lame_mu(), h=h, meta_nx=nx, meta_zs=zs, meta_ys_end=ys_end)


def surface_points(rng, x_range, y_range, z, count):
    """Seeded points uniform on the horizontal rectangle x_range x y_range at
    height z: rest positions (3, count) of embedded collision proxies."""
    x = rng.uniform(x_range[0], x_range[1], count)
    y = rng.uniform(y_range[0], y_range[1], count)
    return np.vstack([x, y, np.full(count, float(z))])


def top_face_proxy_points(scene, count, seed=11):
    """Embedded proxies on the top face of a grid scene: count seeded rest
    positions, uniform over the face (z = nz h)."""
    rng = np.random.default_rng(seed)
    return surface_points(rng, (0.0, scene.nx * scene.h), (0.0, scene.ny * scene.h),
                          scene.nz * scene.h, count)


def region_tets(rest, tets, region, dirichlet):
    """Indices of the tets whose four vertices are free region nodes (the set
    that embeds the proxies)."""
    ok = region & ~dirichlet
    return np.nonzero(np.all(ok[tets], axis=0))[0]


@dataclass
class LevelSetBodies:
    """Rest-pose level sets of the two lips of a slit and the embedded proxies
    on both lip surfaces (all ids global; rest positions (3, *))."""
    proxy_points: np.ndarray   # (3, n_prox) rest positions
    proxy_body: np.ndarray     # (n_prox,) 0 = lower lip, 1 = upper lip
    body_tets: np.ndarray      # (4, n_cand) global node ids
    body_phi: np.ndarray       # (4, n_cand) signed distance to the lip plane (< 0 inside)
    body_id: np.ndarray        # (n_cand,)


def slit_levelset_bodies(sc, per_cell=1.0, seed=15):
    """Lip bodies of a slit scene for rest-pose level-set self-collision: the
    region tets below the slit plane (body 0) and above it (body 1); the signed
    distance of each body's rest shape near the slit is the distance to the
    plane z = zs (negative inside the body), given at each tet corner.  Proxies:
    per_cell seeded points per lip cell face, uniform over the slit footprint
    on each lip."""
    zs = float(sc.meta_zs) * sc.h
    sel = region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)
    T = sc.tets[:, sel]
    zc = sc.rest[2][T].mean(axis=0)
    body = (zc > zs).astype(np.int32)
    Z = sc.rest[2][T]
    phi = np.where(body[None, :] == 1, zs - Z, Z - zs)
    rng = np.random.default_rng(seed)
    nfx, nfy = sc.meta_nx, sc.meta_ys_end
    count = int(round(per_cell * nfx * nfy))
    lo = surface_points(rng, (0.0, nfx * sc.h), (0.0, nfy * sc.h), zs, count)
    up = surface_points(rng, (0.0, nfx * sc.h), (0.0, nfy * sc.h), zs, count)
    pts = np.concatenate([lo, up], axis=1)
    pb = np.concatenate([np.zeros(count, np.int32), np.ones(count, np.int32)])
    return LevelSetBodies(proxy_points=pts, proxy_body=pb, body_tets=T.astype(np.int64),
                          body_phi=phi, body_id=body)
