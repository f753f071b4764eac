"""Explicit MPS operators on the GPU (sph_mps_operators) against the oracle,
through the C ABI (needs an MI355X).

* A random cloud with a random scalar field and coincident pairs, a
  dam-break particle set (fluid and walls) with r_e = 2.1 l0 on cells built
  with h = r_e / 2, and a full lattice block: the particle number density,
  the Laplacian and gradient of the field and the centroid deviation within
  1e-12 (FP64 both sides, summation order aside), and the free-surface flags
  identical (except where a criterion sits within rounding of its threshold).
"""
import numpy as np
import pytest

from paper_2306_01959_amd import scene

pytestmark = pytest.mark.gpu

K_MPS = 2.1


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    return lib


def _mps_scene(sc, l0):
    """The same particles with a cell grid of edge r_e (h = r_e / 2)."""
    re = K_MPS * l0
    lo = [min(v.min(), 0.0) - 0.05 for v in (sc.x, sc.y, sc.z)]
    hi = [max(v.max(), 0.0) + 0.05 for v in (sc.x, sc.y, sc.z)]
    prm = scene.make_params(l0, h_factor=re / (2 * l0), lo=lo, hi=hi)
    out = sc.copy()
    out.params = prm
    return out


def _compare(gpu, orc, sc, l0, phi, label):
    re = K_MPS * l0
    n0, lam = orc.mps_lattice(l0, re)
    p = orc.par(sc.params)
    ref = orc.mps_operators(p, sc.x, sc.y, sc.z, phi, re, n0, lam, 0.98, 0.2, l0)
    sim = gpu.Simulation(sc, "fp64")
    got = sim.mps_operators(re, l0, phi=phi)
    pnd, lap, grad, sig, surf = ref
    scale_l = max(np.abs(lap).max(), 1e-300)
    scale_g = max(np.abs(grad).max(), 1e-300)
    e = dict(pnd=np.abs(got["pnd"] - pnd).max() / n0,
             lap=np.abs(got["lap"] - lap).max() / scale_l,
             grad=np.abs(got["grad"] - grad).max() / scale_g,
             sigma=np.abs(got["sigma"] - sig).max() / l0)
    near = (np.abs(pnd - 0.98 * n0) < 1e-9 * n0) | (np.abs(sig - 0.2 * l0) < 1e-9 * l0)
    mism = np.count_nonzero((got["surface"] != surf) & ~near)
    print(f"\n{label}: n={sc.n}, surface {int(surf.sum())}, errors "
          f"{ {k: f'{v:.1e}' for k, v in e.items()} }, flag mismatches {mism}", flush=True)
    for k, v in e.items():
        assert v < 1e-12, (label, k, v)
    assert mism == 0
    return ref


def test_mps_random_cloud(gpu, oracle_lib):
    l0 = 0.01
    sc = scene.random_cloud(6000, 5, dp=l0, box=0.15, boundary_fraction=0.2)
    sc.x[10:20] = sc.x[:10]          # coincident pairs (left out of every sum)
    sc.y[10:20] = sc.y[:10]
    sc.z[10:20] = sc.z[:10]
    rng = np.random.default_rng(9)
    phi = rng.normal(size=sc.n)
    _compare(gpu, oracle_lib, _mps_scene(sc, l0), l0, phi, "random cloud")


def test_mps_dam_break(gpu, oracle_lib):
    l0 = 0.02
    sc = _mps_scene(scene.config_scene(1), l0)
    phi = 1000.0 * 9.81 * (0.3 - sc.z)      # a hydrostatic-like field
    pnd, lap, grad, sig, surf = _compare(gpu, oracle_lib, sc, l0, phi, "dam break")
    f = ~sc.is_boundary
    assert surf[f & (sc.z > 0.29)].mean() > 0.9       # the water's top layer
    assert surf[f & (sc.z < 0.2) & (sc.x > 0.1) & (sc.x < 0.3)].sum() == 0


def test_mps_lattice_block(gpu, oracle_lib):
    l0 = 2.0 ** -7
    k = np.arange(14)
    zz, yy, xx = np.meshgrid(k, k, k, indexing="ij")
    x = 0.125 + xx.ravel() * l0
    y = 0.125 + yy.ravel() * l0
    z = 0.125 + zz.ravel() * l0
    n = x.size
    zero = np.zeros(n)
    sc = scene.Scene("block", x, y, z, zero.copy(), zero.copy(), zero.copy(),
                     np.full(n, 1000.0), np.zeros(n, bool), {})
    sc = _mps_scene(sc, l0)
    c = 0.125 + 6.5 * l0
    phi = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    _, lap, _, _, surf = _compare(gpu, oracle_lib, sc, l0, phi, "lattice block")
    inner = np.max(np.abs(np.stack([x, y, z], 1) - c), axis=1) < 3.0 * l0
    assert np.allclose(lap[inner], 6.0, rtol=1e-11)
    assert surf[z == z.max()].all() and not surf[inner].any()


def test_mps_without_field_and_dense_rows(gpu, oracle_lib):
    """phi = NULL: only the density, the centroid deviation and the flags,
    identical to the run with a field; and a cloud eight times denser than
    l0^-3, whose waves' stencil rows hold more candidates than one staging
    buffer (they load from memory instead), against the oracle."""
    l0 = 0.02
    sc = _mps_scene(scene.config_scene(1), l0)
    re = K_MPS * l0
    n0, lam = oracle_lib.mps_lattice(l0, re)
    sim = gpu.Simulation(sc, "fp64")
    with_phi = sim.mps_operators(re, l0, phi=np.asarray(sc.z, np.float64))
    without = sim.mps_operators(re, l0, phi=None)
    assert "lap" not in without and "grad" not in without
    for k in ("pnd", "sigma", "surface"):
        assert np.array_equal(without[k], with_phi[k]), k
    ref = oracle_lib.mps_operators(oracle_lib.par(sc.params), sc.x, sc.y, sc.z, None, re, n0,
                                   lam, 0.98, 0.2, l0)
    assert np.abs(without["pnd"] - ref[0]).max() < 1e-12 * n0
    assert np.abs(without["sigma"] - ref[3]).max() < 1e-12 * l0
    # dense: ~74 particles per cell of edge r_e, so a wave's row range of
    # three or four cells holds about 220-300 candidates, either side of 256
    l0 = 0.01
    dense = scene.random_cloud(8000, 11, dp=l0, box=0.1)
    _compare(gpu, oracle_lib, _mps_scene(dense, l0), l0,
             np.random.default_rng(3).normal(size=dense.n), "dense cloud")
