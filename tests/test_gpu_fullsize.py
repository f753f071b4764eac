"""Parity at the workloads' full sizes, in the launch shapes the benchmark
uses (the autotuner's table), through the C ABI.

* Obstacle dam break at dp = 0.005 (875,904 particles) and dp = 0.0025
  (5,798,336 particles): rates of every particle at a state the oracle
  produced (a few oracle steps from the initial set), against the oracle's
  rates at that state: mixed <= 1e-5 relative L2 (the interaction-only
  norm too), FP64 <= 1e-12 (interaction-only 1e-11); interacting pair counts
  equal to the oracle's in FP64.  The achieved errors are printed.
* The 64-instance ensemble (4,526,960 particles): every instance's rates
  against the oracle at its own oracle-advanced state; the lagged, fused,
  graph-replayed run equal bit for bit to eager launches of the same steps.
"""
import numpy as np
import pytest

from paper_2306_01959_amd import autotune, scene
from tests.gpu_helpers import rel_l2, scene_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    return lib


def table_shape(precision, sc):
    """Apply the autotuner table's interaction shape for (precision, sc), the
    shape the benchmark runs it in."""
    tab = autotune._load()
    d = sc.params["dims"]
    ent = tab.get(f"{precision}:n={sc.n}:dims={d[0]}x{d[1]}x{d[2]}")
    if ent is not None:
        autotune.apply(precision, ent["shape"])
    return ent


def oracle_state(orc, sc, nsteps):
    p = orc.par(sc.params)
    st = orc.State(sc)
    orc.run(p, st, nsteps, dt_mode=1)
    return p, st


def check_rates(gpu, orc, sc, p, st, precision):
    cur, prev = scene_from_oracle(st, sc.params)
    ref_r, ref_cnt = orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd,
                               want_counts=True)
    sim = gpu.Simulation(cur, precision)
    sim.upload(cur, prev)
    d0, _ = sim.diagnostics()
    got = sim.rates_by_id()
    d1, _ = sim.diagnostics()
    tol = 1e-12 if precision == "fp64" else 1e-5
    errs = [rel_l2(got[k], ref_r[k]) for k in range(5)]
    # interaction-only norm: gravity removed from the fluid accelerations
    f = ~cur.is_boundary
    g = np.asarray(sc.params["g"])
    a_got = np.concatenate([got[k][f] - g[k] for k in range(3)])
    a_ref = np.concatenate([ref_r[k][f] - g[k] for k in range(3)])
    e_int = rel_l2(a_got, a_ref)
    print(f"\n{sc.name} ({sc.n} particles) {precision}: rel L2 ax {errs[0]:.2e} ay "
          f"{errs[1]:.2e} az {errs[2]:.2e} drho {errs[3]:.2e} mumax {errs[4]:.2e}, "
          f"interaction-only {e_int:.2e}", flush=True)
    for k in range(4):
        assert errs[k] < tol, (precision, k, errs[k])
    assert e_int < (1e-11 if precision == "fp64" else 1e-5)
    if precision == "fp64":
        pairs = [d1[k] - d0[k] for k in ("pairs_ff", "pairs_fb", "pairs_bf")]
        assert pairs == [int(c) for c in ref_cnt], (pairs, ref_cnt)
    del sim


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_obstacle_dp0005_rates(gpu, oracle_lib, precision):
    sc = scene.config_scene(3)
    assert sc.n == 875904
    p, st = oracle_state(oracle_lib, sc, 8)
    try:
        table_shape(precision, sc)
        check_rates(gpu, oracle_lib, sc, p, st, precision)
    finally:
        gpu.set_tuning()


@pytest.fixture(scope="module")
def config5_state(oracle_lib):
    sc = scene.config_scene(5)
    assert sc.n == 5798336
    p, st = oracle_state(oracle_lib, sc, 2)
    return sc, p, st


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_obstacle_dp00025_rates(gpu, oracle_lib, config5_state, precision):
    """The headline workload in both precisions, in the benchmark's launch
    shape for it (FP64 pair counts equal to the oracle's)."""
    sc, p, st = config5_state
    try:
        table_shape(precision, sc)
        check_rates(gpu, oracle_lib, sc, p, st, precision)
    finally:
        gpu.set_tuning()


@pytest.fixture(scope="module")
def ensemble_scenes():
    scs = scene.ensemble(64)
    assert sum(s.n for s in scs) == 4526960
    return scs


def test_ensemble_fullsize_rates(gpu, oracle_lib, ensemble_scenes):
    """Every instance of the 64-instance batch, two oracle steps in, in the
    batch's tuned launch shape."""
    orc = oracle_lib
    cur, states = [], []
    for sc in ensemble_scenes:
        p, st = oracle_state(orc, sc, 2)
        c, _ = scene_from_oracle(st, sc.params)
        cur.append(c)
        states.append((p, st))
    ens = gpu.Ensemble(cur, "mixed")
    try:
        tab = autotune._load()
        ent = tab.get(f"ensemble:mixed:n={ens.n}:inst={ens.ninst}")
        if ent is not None:
            autotune.apply("mixed", ent["shape"])
        got = ens.rates_by_id()
    finally:
        gpu.set_tuning()
    worst = 0.0
    for k, (p, st) in enumerate(states):
        ref = orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd)
        o, c = ens.offsets[k], ens.counts[k]
        for q in range(4):
            worst = max(worst, rel_l2(got[q][o:o + c], ref[q]))
    assert worst < 1e-5, worst


def test_ensemble_fullsize_graph_equals_eager(gpu, ensemble_scenes):
    """80 steps of the benchmark's ensemble form (lagged dt, fused update):
    2 eager, then a 40-step graph replayed once, then 38 eager, against 80
    eager steps."""
    import torch
    a = gpu.Ensemble(ensemble_scenes, "mixed")
    a.run(80, -1.0, 0, mode=gpu.RUN_LAGGED)
    ra = a.fetch()
    da = a.diagnostics()
    del a
    b = gpu.Ensemble(ensemble_scenes, "mixed", stream=torch.cuda.Stream())
    b.run(80, -1.0, 0, mode=gpu.RUN_LAGGED | gpu.RUN_GRAPH)
    rb = b.fetch()
    db = b.diagnostics()
    for key in ("x", "y", "z", "ux", "uz", "rho"):
        assert np.array_equal(ra[key], rb[key]), key
    for k in range(len(ensemble_scenes)):
        assert da[k]["time"] == db[k]["time"]
        assert da[k]["n_nonfinite"] == 0
        assert da[k]["flags"] & gpu.FLAG_DT_CFL == 0


def test_obstacle_dp00025_long_run(gpu):
    """The headline workload's full 2000 steps (mixed, device-side time step,
    the benchmark's launch shape), diagnostics every 100 steps: the mass is
    the same bit for bit every time, nothing leaves the grid or turns
    non-finite, no step exceeds its time-step bound, the total energy
    (kinetic + potential + internal) stays within 2 % of its start, and the
    surge front advances as the column collapses."""
    sc = scene.config_scene(5)
    try:
        table_shape("mixed", sc)
        sim = gpu.Simulation(sc, "mixed")
        d0, _ = sim.diagnostics()
        e0 = d0["e_kin"] + d0["e_pot"] + d0["e_int"]
        fronts = [d0["x_front"]]
        for k in range(20):
            sim.run(100, -1.0, 100 * k)
            d, _ = sim.diagnostics()
            e = d["e_kin"] + d["e_pot"] + d["e_int"]
            fronts.append(d["x_front"])
            assert d["mass"] == d0["mass"] and d["n"] == d0["n"]
            assert d["n_nonfinite"] == 0 and d["n_outside"] == 0
            assert d["flags"] & gpu.FLAG_DT_CFL == 0
            assert abs(e - e0) <= 0.02 * abs(e0), (k, e, e0)
        print(f"\nconfiguration 5, 2000 mixed steps: t = {d['time']:.4f} s, front "
              f"{fronts[0]:.3f} -> {fronts[-1]:.3f} m, energy {e0:.3f} -> {e:.3f} J, "
              f"max |u| {d['umax']:.3f} m/s", flush=True)
        assert fronts[-1] > fronts[0] + 0.05
        assert np.all(np.diff(fronts) >= -1e-9)
    finally:
        gpu.set_tuning()


def test_ensemble_long_run(gpu, ensemble_scenes):
    """The 64-instance batch's 500 steps in the benchmark's form (lagged dt,
    fused update, graph replays): every instance keeps its mass bit for bit,
    stays finite and in its grid, never steps past its lagged bound, does not
    gain total energy (viscosity up to alpha = 0.1 dissipates some: a loss of
    at most 10 %) and moves its front downstream."""
    import torch
    ens = gpu.Ensemble(ensemble_scenes, "mixed", stream=torch.cuda.Stream())
    try:
        tab = autotune._load()
        ent = tab.get(f"ensemble:mixed:n={ens.n}:inst={ens.ninst}")
        if ent is not None:
            autotune.apply("mixed", ent["shape"])
        d0 = ens.diagnostics()
        ens.run(40, -1.0, 0, mode=gpu.RUN_LAGGED)
        ens.run(480, -1.0, 40, mode=gpu.RUN_LAGGED | gpu.RUN_GRAPH)
        d1 = ens.diagnostics()
    finally:
        gpu.set_tuning()
    rel = []
    for a, b in zip(d0, d1):
        assert b["mass"] == a["mass"] and b["n"] == a["n"]
        assert b["n_nonfinite"] == 0 and b["n_outside"] == 0
        assert b["flags"] & gpu.FLAG_DT_CFL == 0
        ea = a["e_kin"] + a["e_pot"] + a["e_int"]
        eb = b["e_kin"] + b["e_pot"] + b["e_int"]
        rel.append((eb - ea) / abs(ea))
        assert b["x_front"] > a["x_front"]
    rel = np.array(rel)
    print(f"\nensemble, 520 steps: relative energy change {rel.min():.2e} .. {rel.max():.2e}",
          flush=True)
    assert rel.max() < 1e-3 and rel.min() > -0.1
