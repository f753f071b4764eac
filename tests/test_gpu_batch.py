"""Batched ensembles (sph_batch_*) on the GPU, through the C ABI.

An ensemble is several independent dam breaks with their own spacing, grid
and alpha (the artificial-viscosity study of Section 4 run as one batch).
Every instance of a batch must behave exactly like the same system run
alone: the batch path is compared bit for bit with the single-system path at
the same launch shape, and each instance with the FP64 oracle (FP64 path
1e-12 relative L2, mixed path 1e-5 on rates).  The lagged-dt fused step and
the graph replays are compared with the oracle's lagged-dt run and with the
eager launches.
"""
import numpy as np
import pytest

from paper_2306_01959_amd import scene
from tests.gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

DPS = (0.04, 0.05, 0.06)
N_INST = 4


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    return lib


@pytest.fixture
def shape(gpu):
    """A fixed launch shape for both paths, restored afterwards."""
    gpu.set_tuning(3, 3, 16, 16)
    yield
    gpu.set_tuning(0, 0, 0, 0)


@pytest.fixture(scope="module")
def scenes():
    return scene.ensemble(N_INST, master_seed=11, dps=DPS)


@pytest.fixture(scope="module")
def developed(oracle_lib, scenes):
    """Each instance advanced 30 oracle steps: (scene of the current level,
    oracle state)."""
    orc = oracle_lib
    out = []
    for sc in scenes:
        p = orc.par(sc.params)
        st = orc.State(sc)
        orc.run(p, st, 30, dt_mode=1)
        cur = scene.Scene(sc.name, st.x.copy(), st.y.copy(), st.z.copy(), st.ux.copy(),
                          st.uy.copy(), st.uz.copy(), st.rho.copy(), sc.is_boundary.copy(),
                          dict(sc.params))
        out.append((cur, st))
    return out


def test_instances_are_uneven(scenes):
    counts = [s.n for s in scenes]
    assert len(set(counts)) > 1
    alphas = [s.params["alpha"] for s in scenes]
    assert len(set(alphas)) == len(alphas)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_cells_partition(gpu, scenes, precision):
    ens = gpu.Ensemble(scenes, precision)
    ens.build_cells()
    ens.sync()
    ids = ens.ids()
    assert np.array_equal(np.sort(ids), np.arange(ens.n))
    inst = np.searchsorted(ens.offsets, ids, side="right") - 1
    # instances occupy consecutive ranges in instance order
    assert np.all(np.diff(inst) >= 0)
    for k, sc in enumerate(scenes):
        sel = inst == k
        assert sel.sum() == sc.n
        loc = ids[sel] - ens.offsets[k]
        x = ens._cur("x").cpu().numpy()[sel]
        assert np.array_equal(x, sc.x[loc])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_rates_equal_single(gpu, shape, developed, precision):
    scs = [d[0] for d in developed]
    ens = gpu.Ensemble(scs, precision)
    got = ens.rates_by_id()
    for k, sc in enumerate(scs):
        ref = gpu.Simulation(sc, precision).rates_by_id()
        o, c = ens.offsets[k], ens.counts[k]
        for q in range(5):
            assert np.array_equal(got[q][o:o + c], ref[q]), (k, q)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batch_rates_vs_oracle(gpu, oracle_lib, developed, precision, tol):
    orc = oracle_lib
    scs = [d[0] for d in developed]
    ens = gpu.Ensemble(scs, precision)
    got = ens.rates_by_id()
    for k, (sc, st) in enumerate(developed):
        p = orc.par(sc.params)
        ref = orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd)
        o, c = ens.offsets[k], ens.counts[k]
        for q in range(4):
            err = rel_l2(got[q][o:o + c], ref[q])
            assert err < tol, (k, q, err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_run_equals_single(gpu, shape, scenes, precision):
    ens = gpu.Ensemble(scenes, precision)
    ens.run(12, -1.0, 0)
    got = ens.fetch()
    dg = ens.diagnostics()
    for k, sc in enumerate(scenes):
        sim = gpu.Simulation(sc, precision)
        sim.run(12, -1.0, 0)
        ref = sim.fetch()
        d1, _ = sim.diagnostics()
        o, c = ens.offsets[k], ens.counts[k]
        for key in ("x", "y", "z", "ux", "uz", "rho", "rhom"):
            assert np.array_equal(got[key][o:o + c], ref[key]), (k, key)
        assert dg[k]["time"] == d1["time"]
        assert dg[k]["dt_last"] == d1["dt_last"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_more_than_64_instances(gpu, shape, precision):
    """70 instances: the chunk-list kernels find a half-row's instance 64
    instances at a time, so half-rows of the instances past the first 64 take
    a second round; the first, the 64th and the last instance each equal the
    same system run alone."""
    scs = scene.ensemble(70, master_seed=5, dps=DPS)
    ens = gpu.Ensemble(scs, precision)
    ens.run(6, -1.0, 0)
    got = ens.fetch()
    for k in (0, 63, 64, 69):
        sim = gpu.Simulation(scs[k], precision)
        sim.run(6, -1.0, 0)
        ref = sim.fetch()
        o, c = ens.offsets[k], ens.counts[k]
        for key in ("x", "y", "z", "ux", "uz", "rho"):
            assert np.array_equal(got[key][o:o + c], ref[key]), (k, key)


def test_batch_lagged_fp64_vs_oracle(gpu, oracle_lib, scenes):
    """45 fused steps with the lagged CFL dt (crossing the Euler reset at
    step 40) against the oracle's lagged-dt run of every instance."""
    orc = oracle_lib
    ens = gpu.Ensemble(scenes, "fp64")
    ens.run(45, -1.0, 0, mode=gpu.RUN_LAGGED)
    got = ens.fetch()
    dg = ens.diagnostics()
    for k, sc in enumerate(scenes):
        p = orc.par(sc.params)
        st = orc.State(sc)
        dts, _ = orc.run(p, st, 45, dt_mode=2)
        o, c = ens.offsets[k], ens.counts[k]
        for key, ref in (("ux", st.ux), ("uz", st.uz)):
            err = rel_l2(got[key][o:o + c], ref)
            assert err < 1e-10, (k, key, err)
        assert rel_l2(got["rho"][o:o + c] - 1000.0, st.rho - 1000.0) < 1e-10
        assert np.abs(got["x"][o:o + c] - st.x).max() < 1e-9 * sc.params["dp"]
        assert abs(dg[k]["time"] - dts.sum()) <= 1e-12 * dts.sum()
        assert abs(dg[k]["dt_last"] - dts[-1]) <= 1e-12 * dts[-1]
    assert not (dg[0]["flags"] & gpu.FLAG_DT_CFL)


def test_batch_lagged_mixed_fixed_dt_vs_oracle(gpu, oracle_lib, scenes):
    orc = oracle_lib
    dt = 2.0e-4
    ens = gpu.Ensemble(scenes, "mixed")
    ens.run(45, dt, 0, mode=gpu.RUN_LAGGED)
    got = ens.fetch()
    for k, sc in enumerate(scenes):
        p = orc.par(sc.params)
        st = orc.State(sc)
        orc.run(p, st, 45, dt_mode=0, dt_in=np.full(45, dt))
        o, c = ens.offsets[k], ens.counts[k]
        for key, ref in (("ux", st.ux), ("uz", st.uz)):
            err = rel_l2(got[key][o:o + c], ref)
            assert err < 1e-4, (k, key, err)
        assert np.abs(got["x"][o:o + c] - st.x).max() < 1e-5 * sc.params["dp"]


@pytest.mark.parametrize("mode", ["lagged", "plain"])
def test_graph_replay_equals_eager(gpu, scenes, mode):
    """100 steps: 2 eager, then a 40-step graph replayed twice, then 18
    eager; bit-identical to 100 eager steps."""
    import torch
    base = gpu.RUN_LAGGED if mode == "lagged" else 0
    a = gpu.Ensemble(scenes, "mixed")
    a.run(100, -1.0, 0, mode=base)
    ra = a.fetch()
    b = gpu.Ensemble(scenes, "mixed", stream=torch.cuda.Stream())
    b.run(100, -1.0, 0, mode=base | gpu.RUN_GRAPH)
    rb = b.fetch()
    for key in ra:
        assert np.array_equal(ra[key], rb[key]), key
    da, db = a.diagnostics(), b.diagnostics()
    for k in range(len(scenes)):
        assert da[k]["time"] == db[k]["time"]
        assert da[k]["steps"] == db[k]["steps"] == 100


def test_batch_diagnostics_vs_oracle(gpu, oracle_lib, developed):
    orc = oracle_lib
    scs = [d[0] for d in developed]
    ens = gpu.Ensemble(scs, "fp64")
    dg = ens.diagnostics()
    for k, (sc, st) in enumerate(developed):
        ref = orc.diagnostics(orc.par(sc.params), st)
        assert dg[k]["n"] == sc.n
        assert abs(dg[k]["mass"] - ref["mass"]) <= 1e-12 * ref["mass"]
        assert abs(dg[k]["e_kin"] - ref["e_kin"]) <= 1e-12 * ref["e_kin"]
        assert abs(dg[k]["e_pot"] - ref["e_pot"]) <= 1e-12 * abs(ref["e_pot"])
        assert abs(dg[k]["umax"] - ref["umax"]) <= 1e-12 * ref["umax"]
        assert dg[k]["x_front"] == ref["x_front"]


def test_lagged_step_without_bound_is_flagged(gpu, scenes):
    """A lagged step n > 0 on a fresh workspace has no bound to use: it takes
    dt = 0 (nothing moves) and raises the CFL flag."""
    ens = gpu.Ensemble(scenes[:2], "fp64")
    x0 = ens.fetch()["x"]
    ens.run(1, -1.0, 5, mode=gpu.RUN_LAGGED)
    out = ens.fetch()
    assert np.array_equal(out["x"], x0)
    dg = ens.diagnostics()
    assert dg[0]["flags"] & gpu.FLAG_DT_CFL
    assert dg[0]["dt_last"] == 0.0


def test_fused_step_counts_feed_the_sort(gpu):
    """The lagged fused row-split interaction (groups of 16) writes the next
    sort's keys and counts their first digits per sort tile, so the sort after
    it launches no histogram of its own.  That sort's order must be the stable
    sort, by cell key, of the positions the fused step left, in the order
    before it: each instance's fluid then its boundary particles, cell row by
    cell row, cell x by cell x (step 5 is no refresh: no sub-cell bits)."""
    from tests import bruteforce
    scenes = scene.ensemble(6, master_seed=31, dps=(0.02, 0.015))
    gpu.set_tuning(kernel_mixed=1, split_mixed=1, group_mixed=16)
    try:
        a = gpu.Ensemble(scenes, "mixed")
        a.run(5, -1.0, 0, mode=gpu.RUN_LAGGED)   # steps 1..4 fused
        ids_a = a.ids()
        x = a._cur("x").cpu().numpy()
        y = a._cur("y").cpu().numpy()
        z = a._cur("z").cpu().numpy()
        b = gpu.Ensemble(scenes, "mixed")
        b.run(6, -1.0, 0, mode=gpu.RUN_LAGGED)   # step 5 sorts what step 4 counted
        ids_b = b.ids()
    finally:
        gpu.set_tuning()
    counts = np.array([s.n for s in scenes])
    offsets = np.concatenate([[0], np.cumsum(counts)[:-1]])
    inst = np.searchsorted(offsets, ids_a, side="right") - 1
    isb = np.concatenate([s.is_boundary for s in scenes])[ids_a]
    key = np.zeros(ids_a.size, np.int64)
    cell_base = 0
    for k, s in enumerate(scenes):
        m = inst == k
        nx, ny, nz = s.params["dims"]
        (cx, cy, cz), _ = bruteforce.cells_and_offsets(x[m], y[m], z[m], s.params["origin"],
                                                       s.params["cell_size"], s.params["dims"])
        key[m] = 2 * cell_base + isb[m] * (nx * ny * nz) + (cy + ny * cz) * nx + cx
        cell_base += nx * ny * nz
    assert np.array_equal(ids_b, ids_a[np.argsort(key, kind="stable")])
