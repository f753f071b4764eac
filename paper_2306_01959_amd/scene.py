"""Seeded synthetic dam-break scenes (input generation only).

This module builds the particle sets that both the HIP library and the CPU
oracle consume.  It holds none of the method's arithmetic: no kernel, no
equation of state, no pair term, no time update.  It only places particles on
lattices, draws the seeded jitter and ensemble parameters, and fills in the
physical constants that the paper's problem statement takes as inputs.

Geometry (a synthetic stand-in for the paper's 3D dam-break cases, Section 3):
  * open-top tank [0, 1.6] x [0, 0.6] x [0, 0.6] m;
  * water block [0, 0.4] x [0, 0.6] x [0, 0.3] m at x = 0;
  * fluid on the lattice (i + 1/2) dp with floor(L / dp) points per axis and a
    seeded uniform jitter of +-0.01 dp per coordinate;
  * two layers of dynamic boundary particles (Section 2.2, dynamic boundary
    conditions): every unjittered lattice point within 2 dp outside the walls
    and the floor;
  * optional obstacle: a two-layer shell of boundary particles inside the box
    [0.84, 0.96] x [0.24, 0.36] x [0, 0.16] m.

Constants: rho0 = 1000 kg/m^3 and g = 9.81 m/s^2 (Section 3), gamma = 7
(Tait equation, Section 2.2), delta = 0.1 (delta-SPH continuity, Section 2.2),
Cr = 0.2 (Section 3), N_s = 40 (Verlet reset period, Section 2.2),
eta^2 = 0.01 h^2 (Monaghan viscosity).  The scene uses h = 1.2 sqrt(3) dp and
c0 = 10 sqrt(g 0.3); the paper's own runs use 2h = 3 l0 and c0 = 20 sqrt(g H_W),
which :func:`paper_params` returns for the alpha study.  The particle mass is
rho0 dp^3 for fluid and boundary alike (the paper writes only "m").
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

RHO0 = 1000.0
G = 9.81
GAMMA = 7.0
DELTA = 0.1
CFL = 0.2
VERLET_NS = 40
ETA2_COEF = 0.01
TANK = (1.6, 0.6, 0.6)
WATER = (0.4, 0.6, 0.3)
OBSTACLE = ((0.84, 0.96), (0.24, 0.36), (0.0, 0.16))
C0_SCENE = 10.0 * math.sqrt(G * 0.3)
#: slack on the cell edge so that every pair closer than 2h lies in the
#: 27-cell stencil even after rounding of the cell coordinate
CELL_SLACK = 2.0 ** -20


@dataclasses.dataclass
class Scene:
    """One dam-break instance: SoA particle arrays in float64 plus parameters.

    ``is_boundary`` marks dynamic boundary particles.  Arrays are in the
    particle's original order; ``ids`` are 0..n-1.
    """
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    rho: np.ndarray
    is_boundary: np.ndarray
    params: Dict[str, object]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(~self.is_boundary))

    @property
    def n_boundary(self) -> int:
        return int(np.count_nonzero(self.is_boundary))

    def copy(self) -> "Scene":
        return Scene(self.name, self.x.copy(), self.y.copy(), self.z.copy(),
                     self.ux.copy(), self.uy.copy(), self.uz.copy(),
                     self.rho.copy(), self.is_boundary.copy(),
                     dict(self.params))


def grid_for(dp: float, h: float, lo: Sequence[float], hi: Sequence[float]
             ) -> Tuple[Tuple[float, float, float], float, Tuple[int, int, int]]:
    """Cell grid covering [lo, hi] with cell edge 2h(1 + 2^-20)."""
    cs = 2.0 * h * (1.0 + CELL_SLACK)
    dims = tuple(max(1, int(math.ceil((b - a) / cs))) for a, b in zip(lo, hi))
    return (float(lo[0]), float(lo[1]), float(lo[2])), cs, dims  # type: ignore


def make_params(dp: float, *, h_factor: float = 1.2 * math.sqrt(3.0),
                c0: float = C0_SCENE, alpha: float = 0.01,
                delta: float = DELTA, cfl: float = CFL,
                gravity: Sequence[float] = (0.0, 0.0, -G),
                rho0: float = RHO0, gamma: float = GAMMA,
                lo: Optional[Sequence[float]] = None,
                hi: Optional[Sequence[float]] = None) -> Dict[str, object]:
    """Parameter dictionary for one instance (the paper's problem inputs)."""
    h = h_factor * dp
    if lo is None:
        lo = (-2.0 * dp, -2.0 * dp, -2.0 * dp)
    if hi is None:
        hi = (TANK[0] + 2.0 * dp, TANK[1] + 2.0 * dp, 2.0 * TANK[2])
    origin, cs, dims = grid_for(dp, h, lo, hi)
    return dict(dp=dp, h=h, rho0=rho0, c0=c0, gamma=gamma, alpha=alpha,
                delta=delta, g=tuple(float(v) for v in gravity),
                eta2_coef=ETA2_COEF, cfl=cfl, mass=rho0 * dp ** 3,
                verlet_ns=VERLET_NS, origin=origin, cell_size=cs, dims=dims)


def paper_params(l0: float, H_w: float, alpha: float) -> Dict[str, object]:
    """The paper's own WCSPH settings: 2h = 3 l0 and c0 = 20 sqrt(g H_W)
    (Section 3; Tables 1 and 3)."""
    return make_params(l0, h_factor=1.5, c0=20.0 * math.sqrt(G * H_w),
                       alpha=alpha)


def _axis_points(dp: float, lo: float, hi: float) -> np.ndarray:
    """Lattice coordinates (i + 1/2) dp that lie strictly inside (lo, hi)."""
    i0 = int(math.floor(lo / dp - 0.5)) - 1
    i1 = int(math.ceil(hi / dp - 0.5)) + 1
    c = (np.arange(i0, i1 + 1, dtype=np.float64) + 0.5) * dp
    return c[(c > lo) & (c < hi)]


def fluid_block(dp: float, size: Sequence[float], rng: np.random.Generator,
                jitter: float = 0.01, corner: Sequence[float] = (0, 0, 0)
                ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """floor(L/dp) lattice points (i + 1/2) dp per axis, plus uniform jitter
    of +-jitter*dp per coordinate."""
    n = [int(math.floor(L / dp + 1e-9)) for L in size]
    ax = [corner[k] + (np.arange(n[k], dtype=np.float64) + 0.5) * dp
          for k in range(3)]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    x, y, z = xx.ravel(), yy.ravel(), zz.ravel()
    if jitter:
        j = rng.uniform(-jitter * dp, jitter * dp, size=(3, x.size))
        x, y, z = x + j[0], y + j[1], z + j[2]
    return x, y, z


def tank_walls(dp: float, tank: Sequence[float] = TANK, layers: int = 2
               ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Lattice points within `layers` dp outside the side walls and floor of
    the open-top tank [0,Lx] x [0,Ly] x [0,Lz]."""
    t = layers * dp
    xs = _axis_points(dp, -t, tank[0] + t)
    ys = _axis_points(dp, -t, tank[1] + t)
    zs = _axis_points(dp, -t, tank[2])
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    x, y, z = xx.ravel(), yy.ravel(), zz.ravel()
    inside = ((x > 0) & (x < tank[0]) & (y > 0) & (y < tank[1]) & (z > 0))
    keep = ~inside
    return x[keep], y[keep], z[keep]


def obstacle_shell(dp: float, box=OBSTACLE, layers: int = 2
                   ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Lattice points inside the box within `layers` dp of its side and top
    faces (the box stands on the tank floor)."""
    (x0, x1), (y0, y1), (z0, z1) = box
    t = layers * dp
    xs = _axis_points(dp, x0, x1)
    ys = _axis_points(dp, y0, y1)
    zs = _axis_points(dp, z0, z1)
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    x, y, z = xx.ravel(), yy.ravel(), zz.ravel()
    core = ((x > x0 + t) & (x < x1 - t) & (y > y0 + t) & (y < y1 - t)
            & (z < z1 - t))
    keep = ~core
    return x[keep], y[keep], z[keep]


def hydrostatic_density(z: np.ndarray, H: float, params: Dict[str, object]
                        ) -> np.ndarray:
    """Initial density of a resting column whose Tait pressure equals
    rho0 g (H - z): the initial condition of the settling case."""
    rho0 = float(params["rho0"])
    gamma = float(params["gamma"])
    c0 = float(params["c0"])
    gmag = abs(float(params["g"][2]))
    B = rho0 * c0 * c0 / gamma
    p = rho0 * gmag * np.maximum(H - z, 0.0)
    return rho0 * np.power(1.0 + p / B, 1.0 / gamma)


def wetted_boundary_density(x, y, z, params, footprint, H: float
                            ) -> np.ndarray:
    """Hydrostatic density for boundary particles beside or under the water
    column (footprint [x0, x1] x [y0, y1] widened by the two wall layers,
    below the surface H); rho0 elsewhere.  Starting the wall at the
    pressure of the water it holds keeps the column from sinking into it."""
    (x0, x1), (y0, y1) = footprint
    t = 2.0 * float(params["dp"]) + 1e-12
    wet = ((x > x0 - t) & (x < x1 + t) & (y > y0 - t) & (y < y1 + t) & (z < H))
    rho = np.full(x.shape, float(params["rho0"]))
    rho[wet] = hydrostatic_density(z[wet], H, params)
    return rho


def assemble(name: str, fluid, boundary_parts: List, params,
             rho_fluid: Optional[np.ndarray] = None,
             wet: Optional[Tuple] = None) -> Scene:
    fx, fy, fz = fluid
    bx = np.concatenate([b[0] for b in boundary_parts]) if boundary_parts else np.zeros(0)
    by = np.concatenate([b[1] for b in boundary_parts]) if boundary_parts else np.zeros(0)
    bz = np.concatenate([b[2] for b in boundary_parts]) if boundary_parts else np.zeros(0)
    x = np.concatenate([fx, bx])
    y = np.concatenate([fy, by])
    z = np.concatenate([fz, bz])
    n = x.size
    isb = np.zeros(n, dtype=bool)
    isb[fx.size:] = True
    rho = np.full(n, float(params["rho0"]))
    if rho_fluid is not None:
        rho[:fx.size] = rho_fluid
    if wet is not None:
        footprint, H = wet
        rho[fx.size:] = wetted_boundary_density(bx, by, bz, params, footprint, H)
    zero = np.zeros(n)
    return Scene(name, x, y, z, zero.copy(), zero.copy(), zero.copy(), rho,
                 isb, dict(params))


def dam_break(dp: float, seed: int, *, alpha: float = 0.01,
              obstacle: bool = False, hydrostatic: bool = False,
              name: Optional[str] = None, **kw) -> Scene:
    """The dam-break scene at spacing dp (the five workload configurations)."""
    params = make_params(dp, alpha=alpha, **kw)
    rng = np.random.Generator(np.random.PCG64(seed))
    fluid = fluid_block(dp, WATER, rng)
    parts = [tank_walls(dp)]
    if obstacle:
        parts.append(obstacle_shell(dp))
    rho_f = None
    wet = None
    if hydrostatic:
        rho_f = hydrostatic_density(fluid[2], WATER[2], params)
        wet = (((0.0, WATER[0]), (0.0, WATER[1])), WATER[2])
    return assemble(name or f"dam_break_dp{dp:g}", fluid, parts, params, rho_f,
                    wet)


#: vertical speed of the gate of the paper's gate-release case (Section 3)
GATE_SPEED = 1.25


def gate_release(dp: float, seed: int, *, alpha: float = 0.01, speed: float = GATE_SPEED,
                 **kw) -> Scene:
    """A gate-release dam break, a stand-in for the paper's force case (its
    geometry figure is not available): the water block of the dam break held
    by a gate, two layers of boundary particles across the tank at
    x in (0.4, 0.4 + 2 dp), y in (0, 0.6), from the floor to 2 dp above the
    water, that moves up at `speed` (1.25 m/s in the paper) from t = 0.  The
    gate particles carry that velocity; everything starts hydrostatic."""
    params = make_params(dp, alpha=alpha, **kw)
    rng = np.random.Generator(np.random.PCG64(seed))
    fluid = fluid_block(dp, WATER, rng)
    x0 = WATER[0]
    xs = _axis_points(dp, x0, x0 + 2.0 * dp)
    ys = _axis_points(dp, 0.0, TANK[1])
    zs = _axis_points(dp, 0.0, WATER[2] + 2.0 * dp)
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    gate = (xx.ravel(), yy.ravel(), zz.ravel())
    rho_f = hydrostatic_density(fluid[2], WATER[2], params)
    sc = assemble(f"gate_dp{dp:g}", fluid, [tank_walls(dp), gate], params, rho_f,
                  (((0.0, WATER[0]), (0.0, WATER[1])), WATER[2]))
    ng = gate[0].size
    sc.uz[sc.n - ng:] = speed
    return sc


def resting_column(dp: float, seed: int, *, tank=(0.2, 0.2, 0.4),
                   H: float = 0.3, alpha: float = 0.1, jitter: float = 0.0,
                   **kw) -> Scene:
    """Water column of height H at rest in a closed-floor tank, initialised
    hydrostatically (the settling case)."""
    lo = (-2.0 * dp, -2.0 * dp, -2.0 * dp)
    hi = (tank[0] + 2.0 * dp, tank[1] + 2.0 * dp, tank[2])
    c0 = kw.pop("c0", 10.0 * math.sqrt(G * H))
    params = make_params(dp, alpha=alpha, c0=c0, lo=lo, hi=hi, **kw)
    rng = np.random.Generator(np.random.PCG64(seed))
    fluid = fluid_block(dp, (tank[0], tank[1], H), rng, jitter=jitter)
    walls = tank_walls(dp, tank)
    rho_f = hydrostatic_density(fluid[2], H, params)
    wet = (((0.0, tank[0]), (0.0, tank[1])), H)
    return assemble(f"column_dp{dp:g}", fluid, [walls], params, rho_f, wet)


def random_cloud(n: int, seed: int, *, dp: float = 0.02, box: float = 0.2,
                 boundary_fraction: float = 0.0, speed: float = 0.0,
                 drho: float = 0.0, **kw) -> Scene:
    """Uniform random cloud in a cube (property tests).  Optional random
    velocities of scale `speed` and density perturbations of scale `drho`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = (-0.05, -0.05, -0.05)
    hi = (box + 0.05, box + 0.05, box + 0.05)
    params = make_params(dp, lo=lo, hi=hi, **kw)
    p = rng.uniform(0.0, box, size=(3, n))
    isb = rng.uniform(size=n) < boundary_fraction
    u = rng.normal(0.0, 1.0, size=(3, n)) * speed
    u[:, isb] = 0.0
    rho = float(params["rho0"]) + rng.uniform(-drho, drho, size=n)
    return Scene(f"cloud{n}", p[0].copy(), p[1].copy(), p[2].copy(),
                 u[0].copy(), u[1].copy(), u[2].copy(), rho, isb, params)


def ensemble(n_instances: int = 64, master_seed: int = 4,
             dps: Sequence[float] = (0.02, 0.015, 0.01),
             alpha_range: Tuple[float, float] = (0.0, 0.1)) -> List[Scene]:
    """Ensemble of independent dam-break instances with drawn dp and alpha
    (the paper's artificial-viscosity study run as a batch)."""
    children = np.random.SeedSequence(master_seed).spawn(n_instances)
    out = []
    for k, ss in enumerate(children):
        rng = np.random.Generator(np.random.PCG64(ss))
        dp = float(dps[int(rng.integers(0, len(dps)))])
        alpha = float(rng.uniform(*alpha_range))
        seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(dam_break(dp, seed, alpha=alpha, name=f"inst{k}"))
    return out


#: artificial viscosities of the paper's study (Table 1; Table 3 uses the
#: first three)
PAPER_ALPHAS = (0.1, 0.01, 0.001, 0.0001)


def viscosity_label(params: Dict[str, object]) -> float:
    """The kinematic viscosity nu0 = alpha h c0 / (2 (dim + 2)) that the paper
    pairs with an artificial viscosity alpha (eq. visc0, dim = 3)."""
    return float(params["alpha"]) * float(params["h"]) * float(params["c0"]) / 10.0


def alpha_study(dp: float = 0.005, alphas: Sequence[float] = PAPER_ALPHAS,
                master_seed: int = 6, obstacle: bool = True) -> List[Scene]:
    """The paper's artificial-viscosity study as an ensemble: one dam break
    (with the obstacle, as in the wave-height and pressure case) per alpha,
    with the paper's own settings, 2h = 3 l0 and c0 = 20 sqrt(g H_W) (H_W =
    0.3 m, the water column), each instance with its own seeded jitter.
    Every scene's name carries its alpha and nu0 (eq. visc0)."""
    children = np.random.SeedSequence(master_seed).spawn(len(alphas))
    out = []
    for a, ss in zip(alphas, children):
        rng = np.random.Generator(np.random.PCG64(ss))
        seed = int(rng.integers(0, 2 ** 31 - 1))
        params = paper_params(dp, WATER[2], a)
        sc_rng = np.random.Generator(np.random.PCG64(seed))
        fluid = fluid_block(dp, WATER, sc_rng)
        parts = [tank_walls(dp)]
        if obstacle:
            parts.append(obstacle_shell(dp))
        name = f"alpha{a:g}_nu{viscosity_label(params):.1e}_dp{dp:g}"
        out.append(assemble(name, fluid, parts, params))
    return out


#: the five workload configurations: (dp, precision, steps, alpha, seed,
#: obstacle, hydrostatic)
CONFIGS = {
    1: dict(dp=0.02, precision="fp64", steps=200, alpha=0.01, seed=1,
            obstacle=False, hydrostatic=False),
    2: dict(dp=0.01, precision="mixed", steps=1000, alpha=0.01, seed=2,
            obstacle=False, hydrostatic=True),
    3: dict(dp=0.005, precision="mixed", steps=2000, alpha=0.01, seed=3,
            obstacle=True, hydrostatic=False),
    5: dict(dp=0.0025, precision="mixed", steps=2000, alpha=0.01, seed=5,
            obstacle=True, hydrostatic=False),
}

#: probe points on the obstacle's front face (configuration 3)
OBSTACLE_PROBES = np.array([[0.84 - 0.005, 0.3, zz]
                            for zz in (0.02, 0.06, 0.10, 0.14)])


def config_scene(k: int) -> Scene:
    c = CONFIGS[k]
    return dam_break(c["dp"], c["seed"], alpha=c["alpha"],
                     obstacle=c["obstacle"], hydrostatic=c["hydrostatic"],
                     name=f"config{k}")
