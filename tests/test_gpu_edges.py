"""Degenerate and edge cases of the HIP path, through the C ABI, against the
oracle or closed forms: a lone fluid particle (free fall, exact), a lone
boundary particle (nothing changes), every particle in one cell of a 1x1x1
grid, coincident particles (neighbours at r = 0), pairs exactly 2h apart
(outside the strict support), an instance of one particle inside a batch,
and every interaction decomposition on the crowded cell.
"""
import numpy as np
import pytest

from paper_2306_01959_amd import scene
from tests.gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

KERNELS = [(1, 1, 8), (1, 3, 16), (1, 9, 64), (2, 1, 8), (2, 1, 64), (3, 1, 8), (4, 1, 16)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    return lib


def make(x, y, z, isb, prm, u=None, rho=None, name="edge"):
    n = len(x)
    u = np.zeros((3, n)) if u is None else u
    rho = np.full(n, float(prm["rho0"])) if rho is None else rho
    return scene.Scene(name, np.asarray(x, float), np.asarray(y, float), np.asarray(z, float),
                       u[0].copy(), u[1].copy(), u[2].copy(), np.asarray(rho, float),
                       np.asarray(isb, bool), prm)


def oracle_rates(orc, sc):
    p = orc.par(sc.params)
    return orc.rates(p, sc.x, sc.y, sc.z, sc.ux, sc.uy, sc.uz, sc.rho,
                     sc.is_boundary.astype(np.uint8))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lone_fluid_particle_falls_freely(gpu, precision):
    prm = scene.make_params(0.02, lo=(0, 0, 0), hi=(0.5, 0.5, 0.5))
    sc = make([0.25], [0.25], [0.40], [False], prm, u=np.array([[0.3], [-0.1], [0.2]]))
    sim = gpu.Simulation(sc, precision)
    ax, ay, az, dr, mu = sim.rates_by_id()
    # the mixed path adds g in FP32
    g = prm["g"][2] if precision == "fp64" else float(np.float32(prm["g"][2]))
    assert (ax[0], ay[0], az[0], dr[0], mu[0]) == (0.0, 0.0, g, 0.0, 0.0)
    dt = 1e-3
    for k in range(60):  # crosses the Euler reset at step 40
        sim.step(dt, k)
    out = sim.fetch()
    t = 60 * dt
    assert out["x"][0] == pytest.approx(0.25 + 0.3 * t, rel=1e-13)
    assert out["uz"][0] == pytest.approx(0.2 + g * t, rel=1e-12)
    assert out["z"][0] == pytest.approx(0.40 + 0.2 * t + 0.5 * g * t * t, rel=1e-12)
    assert out["rho"][0] == prm["rho0"]


def test_lone_boundary_particle_is_still(gpu):
    prm = scene.make_params(0.02, lo=(0, 0, 0), hi=(0.5, 0.5, 0.5))
    sc = make([0.1], [0.2], [0.3], [True], prm)
    sim = gpu.Simulation(sc, "mixed")
    rates = sim.rates_by_id()
    assert all(r[0] == 0.0 for r in rates)
    sim.run(5, 1e-3, 0)
    out = sim.fetch()
    assert (out["x"][0], out["y"][0], out["z"][0], out["rho"][0]) == (0.1, 0.2, 0.3, 1000.0)


def crowded_cell(seed=3, n=300):
    """Every particle in the one cell of a 1x1x1 grid, random velocities and
    densities, a quarter of them boundary."""
    dp = 0.02
    prm = scene.make_params(dp, lo=(0, 0, 0), hi=(0.05, 0.05, 0.05))
    assert tuple(prm["dims"]) == (1, 1, 1)
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 0.05, size=(3, n))
    isb = rng.uniform(size=n) < 0.25
    u = rng.normal(0, 0.5, size=(3, n))
    u[:, isb] = 0.0
    rho = 1000.0 + rng.uniform(-5, 5, size=n)
    return make(p[0], p[1], p[2], isb, prm, u=u, rho=rho, name="crowded")


@pytest.mark.parametrize("shape", KERNELS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_crowded_single_cell(gpu, oracle_lib, shape, precision, tol):
    sc = crowded_cell()
    ref = oracle_rates(oracle_lib, sc)
    try:
        if precision == "fp64":
            gpu.set_tuning(kernel_fp64=shape[0], split_fp64=shape[1], group_fp64=shape[2])
        else:
            gpu.set_tuning(kernel_mixed=shape[0], split_mixed=shape[1], group_mixed=shape[2])
        got = gpu.Simulation(sc, precision).rates_by_id()
    finally:
        gpu.set_tuning()
    for k in range(4):
        assert rel_l2(got[k], ref[k]) < tol, (shape, k)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coincident_particles(gpu, oracle_lib, precision):
    """Two fluid particles at the same point are neighbours (r = 0 < 2h): the
    gradient vanishes there, the delta term's radial factor does not."""
    prm = scene.make_params(0.02, lo=(0, 0, 0), hi=(0.3, 0.3, 0.3))
    x = [0.15, 0.15, 0.16]
    y = [0.15, 0.15, 0.15]
    z = [0.15, 0.15, 0.15]
    sc = make(x, y, z, [False, False, False], prm, rho=np.array([1001.0, 999.0, 1000.5]))
    ref = oracle_rates(oracle_lib, sc)
    got = gpu.Simulation(sc, precision).rates_by_id()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k in range(4):
        assert rel_l2(got[k], ref[k]) < tol, k
    nf, nb, _ = gpu.Simulation(sc, precision).neighbour_stats()
    assert list(nf) == [2, 2, 2] and list(nb) == [0, 0, 0]


def test_support_boundary_is_exclusive(gpu):
    """Particles exactly 2h apart along an axis (exactly representable
    values) are not neighbours; 2h minus one ulp is."""
    h = 0.25
    prm = scene.make_params(1.0, h_factor=h, lo=(0, 0, 0), hi=(4, 4, 4))
    assert prm["h"] == h
    x = np.array([1.0, 1.5, 2.5, np.nextafter(3.0, 0.0)])
    sc = make(x, np.full(4, 2.0), np.full(4, 2.0), [False] * 4, prm)
    nf, nb, _ = gpu.Simulation(sc, "fp64").neighbour_stats()
    # 1.0-1.5: 0.5 = 2h exactly -> no; 1.5-2.5: 1.0 -> no; 2.5-(3-ulp) < 2h -> yes
    assert list(nf) == [0, 0, 1, 1]


def test_single_particle_instance_in_batch(gpu, oracle_lib):
    """A batch holding a one-particle instance next to a crowded one: each
    instance as if alone."""
    prm = scene.make_params(0.02, lo=(0, 0, 0), hi=(0.5, 0.5, 0.5))
    lone = make([0.25], [0.25], [0.40], [False], prm, u=np.array([[0.3], [0.0], [0.0]]))
    crowd = crowded_cell(seed=5, n=200)
    ens = gpu.Ensemble([lone, crowd, lone], "fp64")
    got = ens.rates_by_id()
    pieces = [ens.split_by_instance(g) for g in got]
    assert pieces[0][0][0] == 0.0 and pieces[2][2][0] == prm["g"][2]
    ref = oracle_rates(oracle_lib, crowd)
    for k in range(4):
        assert rel_l2(pieces[k][1], ref[k]) < 1e-12, k
    for k in range(4):
        assert pieces[k][0][0] == pieces[k][2][0]
