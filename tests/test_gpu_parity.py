"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances: the FP64 path within 1e-12 relative L2 of the oracle; the mixed
FP32 path within 1e-5 relative L2 for accelerations and drho/dt.  Neighbour
sets are compared bit-exactly, each against the brute-force definition taken
in the precision the path decides it in.
"""
import math

import numpy as np
import pytest

from paper_2306_01959_amd import scene
from tests import bruteforce
from tests.gpu_helpers import rel_l2, scene_from_oracle, set_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    return lib


@pytest.fixture(scope="module")
def developed(oracle_lib):
    """Configuration-1 dam break advanced 60 steps by the oracle (CFL dt):
    a state with real flow, pressure and viscosity."""
    orc = oracle_lib
    s = scene.config_scene(1)
    p = orc.par(s.params)
    st = orc.State(s)
    orc.run(p, st, 60, dt_mode=1)
    return s.params, st


def _sim(gpu, sc, precision, prev=None, **kw):
    sim = gpu.Simulation(sc, precision, **kw)
    if prev is not None:
        sim.upload(sc, prev)
    return sim


# ---------------------------------------------------------------- cells

def _sort_keys(sc_or_xyz, prm, isb, full):
    """The library's sort key from FP64 positions: class, cell row, cell x,
    then (full) the upper-half flags along y and x (zero for boundary
    particles)."""
    x, y, z = sc_or_xyz
    (cx, cy, cz), _ = bruteforce.cells_and_offsets(x, y, z, prm["origin"], prm["cell_size"],
                                                   prm["dims"])
    nx, ny, nz = prm["dims"]
    key = isb * (nx * ny * nz) + (cy + ny * cz) * nx + cx
    if not full:
        return key
    ux = bruteforce.upper_half(x, prm["origin"][0], prm["cell_size"], prm["dims"][0])
    uy = bruteforce.upper_half(y, prm["origin"][1], prm["cell_size"], prm["dims"][1])
    return key * 4 + np.where(isb, 0, uy * 2 + ux)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_build_cells_invariants(gpu, precision):
    """sph_build_cells sorts on the full key (class, cell row, cell x, the
    halves of the cell along y and x), stably."""
    s = scene.config_scene(1)
    sim = _sim(gpu, s, precision)
    sim.build_cells()
    sim.sync()
    ids = sim.ids()
    assert np.array_equal(np.sort(ids), np.arange(s.n))
    x = sim._cur("x").cpu().numpy()
    y = sim._cur("y").cpu().numpy()
    z = sim._cur("z").cpu().numpy()
    key = _sort_keys((x, y, z), s.params, s.is_boundary[ids], True)
    assert np.all(np.diff(key) >= 0)
    # stable: particles with equal keys keep the original order
    same = np.diff(key) == 0
    assert np.all(np.diff(ids)[same] > 0)
    # positions travelled with their ids
    assert np.array_equal(x, s.x[ids]) and np.array_equal(z, s.z[ids])


def test_step_between_refreshes_sorts_cells_only(gpu):
    """A step whose index is not a multiple of the refresh period sorts on the
    cell key alone: cells in order, and inside a cell the previous order."""
    s = scene.config_scene(1)
    sim = _sim(gpu, s, "fp64")
    sim.run(1, 1e-5, 1)  # step 1: cells of the uploaded (id) order
    ids = sim.ids()
    assert np.array_equal(np.sort(ids), np.arange(s.n))
    key = _sort_keys((s.x[ids], s.y[ids], s.z[ids]), s.params, s.is_boundary[ids], False)
    assert np.all(np.diff(key) >= 0)
    same = np.diff(key) == 0
    assert np.all(np.diff(ids)[same] > 0)
    # and not by the sub-cell bits (the scene's lattice order is not theirs)
    full = _sort_keys((s.x[ids], s.y[ids], s.z[ids]), s.params, s.is_boundary[ids], True)
    assert not np.all(np.diff(full) >= 0)


def test_build_cells_large_sort(gpu):
    """700k particles: many sort tiles per digit, scanned per digit over the
    tiles, each scatter adding the smaller digits' totals; the order must
    still be the stable sort by the full key."""
    sc = scene.random_cloud(700_000, 3, dp=0.002, box=0.2)
    sim = _sim(gpu, sc, "mixed")
    sim.build_cells()
    sim.sync()
    ids = sim.ids()
    key = _sort_keys((sc.x, sc.y, sc.z), sc.params, sc.is_boundary, True)
    assert np.array_equal(ids, np.argsort(key, kind="stable"))


def test_sort_digit_rows_longer_than_one_scan_span(gpu):
    """17 M particles: more than 4096 sort tiles of 4096 keys, so each digit's
    row of per-tile counts is longer than one block's scan span and its scan
    carries from span to span; the order must be the stable sort by the full
    key."""
    n = 17_000_000
    sc = scene.random_cloud(n, 5, dp=0.002, box=0.6)
    sim = _sim(gpu, sc, "mixed")
    sim.build_cells()
    sim.sync()
    ids = sim.ids()
    key = _sort_keys((sc.x, sc.y, sc.z), sc.params, sc.is_boundary, True)
    assert -(-n // 4096) > 4096
    assert np.array_equal(ids, np.argsort(key, kind="stable"))


@pytest.mark.parametrize("case", ["dambreak_146752", "cloud_2500000"])
def test_sort_of_nearly_sorted_input_with_outliers(gpu, case):
    """Upload order: the stable sort by the full key, then in every aligned
    group of 64 particles the sixth moved to the front.  Lane 0 of a wave
    then holds a larger digit than lane 1, one that recurs a few lanes on
    (the wave's digits decrease once); the order must still be the stable
    sort by the full key.  Both tile sizes of the radix sort (the cloud is
    above the small-array limit)."""
    import dataclasses
    if case.startswith("dambreak"):
        sc = scene.config_scene(2)
    else:
        sc = scene.random_cloud(2_500_000, 4, dp=0.002, box=0.3)
    key = _sort_keys((sc.x, sc.y, sc.z), sc.params, sc.is_boundary, True)
    order = np.argsort(key, kind="stable")
    m = order.size // 64 * 64
    g = order[:m].reshape(-1, 64).copy()
    g[:, :6] = np.roll(g[:, :6], 1, axis=1)  # element 5 first
    perm = np.concatenate([g.ravel(), order[m:]])
    assert np.any(key[perm][0:m:64] > key[perm][1:m:64])
    sp = dataclasses.replace(sc, x=sc.x[perm], y=sc.y[perm], z=sc.z[perm], ux=sc.ux[perm],
                             uy=sc.uy[perm], uz=sc.uz[perm], rho=sc.rho[perm],
                             is_boundary=sc.is_boundary[perm])
    # every radix pass (8-bit digits, least significant first) sees some
    # 64-key wave whose digit decreases from one lane to the next, so the
    # scatter's digit-matching fallback runs in each pass
    assert _decreasing_digit_in_every_pass(key[perm])
    sim = _sim(gpu, sp, "mixed")
    sim.build_cells()
    sim.sync()
    assert np.array_equal(sim.ids(), np.argsort(key[perm], kind="stable"))


def _decreasing_digit_in_every_pass(keys, bits=8):
    """LSD passes over `keys` (input order) as the library runs them: for
    each pass, whether some aligned group of 64 consecutive keys of that
    pass's input holds a digit smaller than its left neighbour's."""
    keys = np.asarray(keys, np.int64)
    order = np.arange(keys.size)
    nbits = max(1, int(keys.max()).bit_length())
    ok = []
    for shift in range(0, nbits, bits):
        d = (keys[order] >> shift) & ((1 << bits) - 1)
        m = d.size // 64 * 64
        w = d[:m].reshape(-1, 64)
        ok.append(bool(np.any(np.diff(w, axis=1) < 0)))
        order = order[np.argsort(d, kind="stable")]
    return all(ok) and len(ok) >= 2


def test_sort_of_update_written_keys_with_outliers(gpu):
    """The sort of a run's second step takes the keys the first step's update
    wrote and the digit counts it took per sort tile (not the positions).
    Make that input nearly sorted with outliers: the first particle of every
    aligned group of 64 (in the first step's order) moves one cell along x
    in the first step, so lane 0 of a wave holds a larger key than lane 1.
    The second step's order must be the stable sort of those keys (cells
    only: step 1 is not a refresh step) of the first step's order."""
    s = scene.dam_break(0.01, 2, alpha=0.0, hydrostatic=True, name="outliers")
    prm = s.params
    order0 = np.argsort(_sort_keys((s.x, s.y, s.z), prm, s.is_boundary, True), kind="stable")
    dt = 1e-4
    lead = order0[::64]
    lead = lead[~s.is_boundary[lead]]       # boundary particles do not move
    s.ux[lead] = prm["cell_size"] / dt       # one cell along x in one step
    a = _sim(gpu, s, "mixed")
    a.run(1, dt, 0)
    a.sync()
    ids_a = a.ids()
    assert np.array_equal(ids_a, order0)
    xa = a._cur("x").cpu().numpy()
    ya = a._cur("y").cpu().numpy()
    za = a._cur("z").cpu().numpy()
    key1 = _sort_keys((xa, ya, za), prm, s.is_boundary[ids_a], False)
    assert np.any(key1[0:key1.size // 64 * 64:64] > key1[1:key1.size // 64 * 64 + 1:64])
    assert _decreasing_digit_in_every_pass(key1)
    b = _sim(gpu, s, "mixed")
    b.run(2, dt, 0)
    b.sync()
    assert np.array_equal(b.ids(), ids_a[np.argsort(key1, kind="stable")])


# ----------------------------------------------------------- neighbours

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", [0, 1])
def test_neighbour_sets_bit_exact(gpu, precision, seed):
    prm = scene.make_params(0.02, lo=(0, 0, 0), hi=(0.5, 0.45, 0.4))
    x, y, z = bruteforce.adversarial_cloud(seed, prm)
    n = x.size
    rng = np.random.default_rng(seed + 10)
    isb = rng.uniform(size=n) < 0.3
    zero = np.zeros(n)
    sc = scene.Scene("adv", x, y, z, zero.copy(), zero.copy(), zero.copy(),
                     np.full(n, 1000.0), isb, prm)
    sim = _sim(gpu, sc, precision)
    nf, nb, hs = sim.neighbour_stats()
    if precision == "fp64":
        ref = bruteforce.pairs_fp64(x, y, z, prm["h"])
    else:
        ref = bruteforce.pairs_mixed(x, y, z, prm["h"], prm["origin"], prm["cell_size"],
                                     prm["dims"])
    rf, rb, rh = set_stats(ref, n, isb)
    assert np.array_equal(nf, rf)
    assert np.array_equal(nb, rb)
    assert np.array_equal(hs, rh)


# ---------------------------------------------------------------- rates

def _oracle_rates(orc, params, st):
    p = orc.par(params)
    return orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_rates_developed_state(gpu, oracle_lib, developed, precision, tol):
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    ref = _oracle_rates(oracle_lib, params, st)
    sim = _sim(gpu, sc, precision, prev)
    got = sim.rates_by_id()
    f = ~sc.is_boundary
    g = np.asarray(params["g"])
    for k in range(3):
        assert rel_l2(got[k], ref[k]) < tol, (k, rel_l2(got[k], ref[k]))
    # interaction-only norm (gravity removed)
    a_got = np.stack([got[k][f] - g[k] for k in range(3)])
    a_ref = np.stack([ref[k][f] - g[k] for k in range(3)])
    assert rel_l2(a_got, a_ref) < tol
    assert rel_l2(got[3], ref[3]) < tol
    assert rel_l2(got[4], ref[4]) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config2_first_steps_lockstep(gpu, oracle_lib, precision):
    """Configuration 2 (dp = 0.01, hydrostatic start): for each of the first
    10 steps, the GPU's rates at its own state against the oracle's rates at
    the oracle's state, both advanced with the oracle's dt sequence."""
    orc = oracle_lib
    s = scene.config_scene(2)
    p = orc.par(s.params)
    st = orc.State(s)
    sim = _sim(gpu, s, precision)
    tol = 1e-12 if precision == "fp64" else 1e-5
    worst = 0.0
    for k in range(10):
        ref = orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd)
        got = sim.rates_by_id()
        for c in range(4):
            worst = max(worst, rel_l2(got[c], ref[c]))
        dt = orc.dt_cfl(p, ref[0], ref[1], ref[2], ref[4], st.is_bnd)
        orc.update(p, st, k % 40 == 0, dt, ref)
        sim.step(dt, k)
    assert worst < tol, worst
    out = sim.fetch()
    scale = s.params["dp"]
    assert np.abs(out["x"] - st.x).max() < (1e-12 if precision == "fp64" else 1e-7) * scale * 100


def test_dt_bound_matches_oracle(gpu, oracle_lib, developed):
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    ref = _oracle_rates(oracle_lib, params, st)
    p = oracle_lib.par(params)
    dt_ref = oracle_lib.dt_cfl(p, ref[0], ref[1], ref[2], ref[4], st.is_bnd)
    for precision, tol in (("fp64", 1e-13), ("mixed", 1e-5)):
        sim = _sim(gpu, sc, precision, prev)
        sim.step(-1.0, 1)     # device CFL time step, Verlet branch
        d, _ = sim.diagnostics()
        assert d["dt_last"] == pytest.approx(dt_ref, rel=tol)
        assert d["dt_cfl"] == pytest.approx(dt_ref, rel=tol)


# ---------------------------------------------------------- trajectories

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trajectory_matches_oracle(gpu, oracle_lib, developed, precision):
    """45 steps (crossing the Euler reset at step 40) with the oracle's dt
    sequence from a developed state."""
    orc = oracle_lib
    params, st0 = developed
    sc, prev = scene_from_oracle(st0, params)
    p = orc.par(params)
    st = orc.State(sc)
    st.uxm, st.uym, st.uzm, st.rhom = (prev["ux"].copy(), prev["uy"].copy(),
                                       prev["uz"].copy(), prev["rho"].copy())
    st.step = 60
    dts, _ = orc.run(p, st, 45, dt_mode=1)
    sim = _sim(gpu, sc, precision, prev)
    for k in range(45):
        sim.step(float(dts[k]), 60 + k)
    out = sim.fetch()
    tol = 1e-10 if precision == "fp64" else 1e-5
    for key, ref in (("ux", st.ux), ("uz", st.uz)):
        assert rel_l2(out[key], ref) < tol, (key, rel_l2(out[key], ref))
    assert rel_l2(out["rho"] - 1000.0, st.rho - 1000.0) < tol
    assert np.abs(out["x"] - st.x).max() < 1e-6 * params["dp"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_equals_step_by_step(gpu, precision):
    """A run of 50 steps (each update writes the next sort's keys, across the
    full-key refresh at step 40) equals 50 single steps (each sort computes
    its keys from the positions), bit for bit."""
    s = scene.config_scene(1)
    a = _sim(gpu, s, precision)
    a.run(50, -1.0, 0)
    b = _sim(gpu, s, precision)
    for k in range(50):
        b.step(-1.0, k)
    ra, rb = a.fetch(), b.fetch()
    for key in ra:
        assert np.array_equal(ra[key], rb[key]), key


def test_determinism_bitwise(gpu):
    s = scene.config_scene(1)
    outs = []
    for _ in range(2):
        sim = _sim(gpu, s, "mixed")
        sim.run(25, -1.0, 0)
        outs.append(sim.fetch())
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


# ----------------------------------------------------------- diagnostics

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_diagnostics_match_oracle(gpu, oracle_lib, developed, precision):
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    sim = _sim(gpu, sc, precision, prev)
    probes = np.array([[0.2, 0.3, 0.05], [0.5, 0.3, 0.02], [1.5, 0.3, 0.5]])
    d, pp = sim.diagnostics(probes)
    p = oracle_lib.par(params)
    od = oracle_lib.diagnostics(p, st)
    op = oracle_lib.probes(p, st, probes)
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert d["mass"] == pytest.approx(od["mass"], rel=1e-12)
    assert d["e_kin"] == pytest.approx(od["e_kin"], rel=tol)
    assert d["e_pot"] == pytest.approx(od["e_pot"], rel=1e-12)
    assert d["e_int"] == pytest.approx(od["e_int"], rel=1e-4 if precision == "mixed" else 1e-10)
    assert d["umax"] == pytest.approx(od["umax"], rel=1e-12)
    assert d["x_front"] == od["x_front"]
    for k, key in enumerate(("px", "py", "pz")):
        assert d["mom"][k] == pytest.approx(od[key], rel=1e-9, abs=1e-12)
    assert d["n_fluid"] == sc.n_fluid and d["n"] == sc.n
    assert d["n_nonfinite"] == 0
    assert np.allclose(pp, op, rtol=1e-6 if precision == "mixed" else 1e-12, atol=1e-9)
    assert pp[2] == 0.0          # dry probe


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_front_and_probe_series_match_oracle(gpu, oracle_lib, precision):
    """Short horizon of the configuration-1 dam break from rest (240 steps,
    the oracle's CFL dt sequence fed to the GPU): the surge front and three
    probe pressures sampled every 12 steps stay within 1 % of each series'
    range of the oracle's."""
    s = scene.config_scene(1)
    p = oracle_lib.par(s.params)
    st = oracle_lib.State(s)
    sim = _sim(gpu, s, precision)
    probes = np.array([[0.2, 0.3, 0.03], [0.45, 0.3, 0.02], [0.3, 0.3, 0.15]])
    ref, got = [], []
    step = 0
    for _ in range(20):
        dts, _ = oracle_lib.run(p, st, 12, dt_mode=1)
        for dt in dts:
            sim.step(float(dt), step)
            step += 1
        od = oracle_lib.diagnostics(p, st)
        ref.append([od["x_front"], *oracle_lib.probes(p, st, probes)])
        d, pp = sim.diagnostics(probes)
        got.append([d["x_front"], *pp])
    ref, got = np.array(ref), np.array(got)
    span = ref.max(axis=0) - ref.min(axis=0)
    assert span[0] > 0.05 and (span[1:] > 100.0).all(), span  # the flow does develop
    err = np.abs(got - ref).max(axis=0)
    assert (err <= 0.01 * span).all(), (err / span)


def test_pair_totals_match_oracle(gpu, oracle_lib, developed):
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    p = oracle_lib.par(params)
    _, cnt = oracle_lib.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd,
                              want_counts=True)
    sim = _sim(gpu, sc, "fp64", prev)
    sim.interact()
    d, _ = sim.diagnostics()
    assert (d["pairs_ff"], d["pairs_fb"], d["pairs_bf"]) == cnt


def test_nan_is_flagged(gpu):
    s = scene.config_scene(1)
    s.rho[5] = float("nan")
    sim = _sim(gpu, s, "fp64")
    d, _ = sim.diagnostics()
    assert d["n_nonfinite"] >= 1 and d["flags"] & gpu.FLAG_NONFINITE


def test_outside_particle_clamped_and_counted(gpu):
    s = scene.config_scene(1)
    s.z[0] = 5.0                       # far above the grid top (1.2 m)
    s.x[1] = -1.0                      # left of the grid
    sim = _sim(gpu, s, "mixed")
    d, _ = sim.diagnostics()
    assert d["n_outside"] == 2 and d["flags"] & gpu.FLAG_OUTSIDE
    sim.run(3, -1.0, 0)
    out = sim.fetch()
    assert np.all(np.isfinite(out["x"])) and out["z"][0] < 5.0


# ------------------------------------------------------------ hydrostatics

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hydrostatic_column(gpu, precision):
    """The settling case of the oracle pins, on the GPU path."""
    s = scene.resting_column(0.02, 0, tank=(0.2, 0.2, 0.4), H=0.3, alpha=0.1, delta=0.0)
    sim = _sim(gpu, s, precision)
    h, c0, H = s.params["h"], s.params["c0"], 0.3
    dt = s.params["cfl"] * h / c0
    sim.run(int(0.6 / dt), -1.0, 0)
    zs = np.array([2 * h + 0.001, 0.1, 0.15, 0.2, H - 2 * h])
    d, pp = sim.diagnostics([[0.1, 0.1, zz] for zz in zs])
    err = (pp - 1000.0 * 9.81 * (H - zs)) / (1000.0 * 9.81 * H)
    assert np.abs(err).max() < 0.01, err
    assert d["umax"] < 0.1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_launch_shape_matches(gpu, oracle_lib, developed, precision):
    """Every launch shape the autotuner may pick -- the row-split kernel with
    1, 3 or 9 waves per chunk x 8, 16 or 64 targets per group, the
    group-per-wave kernel with 8, 16 or 64, the cooperative kernel with 8 or
    16 -- gives bit-identical neighbour sets and oracle-parity rates."""
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    ref = _oracle_rates(oracle_lib, params, st)
    tol = 1e-12 if precision == "fp64" else 1e-5
    shapes = [(gpu.SPH_KERNEL_ROWS, split, group) for split in (1, 3, 9)
              for group in (8, 16, 64)]
    shapes += [(gpu.SPH_KERNEL_GROUPS, 1, group) for group in (8, 16, 64)]
    shapes += [(k, 1, group) for k in (gpu.SPH_KERNEL_COOP, gpu.SPH_KERNEL_COOP2)
               for group in (8, 16)]
    stats = []
    try:
        for kernel, split, group in shapes:
            if precision == "fp64":
                gpu.set_tuning(split_fp64=split, group_fp64=group, kernel_fp64=kernel)
            else:
                gpu.set_tuning(split_mixed=split, group_mixed=group, kernel_mixed=kernel)
            sim = _sim(gpu, sc, precision, prev)
            assert gpu.get_split(sim.params, sim.n) == (split, group, kernel)
            got = sim.rates_by_id()
            for k in range(4):
                assert rel_l2(got[k], ref[k]) < tol, (kernel, split, group, k)
            stats.append(sim.neighbour_stats())
    finally:
        gpu.set_tuning()
    for s_ in stats[1:]:
        for a_, b_ in zip(s_, stats[0]):
            assert np.array_equal(a_, b_)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_xcd_run_order_is_bitwise_neutral(gpu, developed, precision):
    """The order in which workgroups take chunks (runs of 1, 8 or 32 chunks
    per XCD) changes no result bit: each chunk's sums are its own.  Row-split
    and group-per-wave kernels."""
    params, st = developed
    sc, prev = scene_from_oracle(st, params)
    try:
        for kernel, split, group in ((gpu.SPH_KERNEL_ROWS, 1, 16), (gpu.SPH_KERNEL_GROUPS, 1, 8),
                                     (gpu.SPH_KERNEL_COOP, 1, 16)):
            outs = []
            for run in (1, 8, 32):
                if precision == "fp64":
                    gpu.set_tuning(split_fp64=split, group_fp64=group, kernel_fp64=kernel,
                                   xcd_run_fp64=run)
                else:
                    gpu.set_tuning(split_mixed=split, group_mixed=group, kernel_mixed=kernel,
                                   xcd_run_mixed=run)
                sim = _sim(gpu, sc, precision, prev)
                outs.append(sim.rates_by_id())
            for o in outs[1:]:
                for k in range(len(o)):
                    assert np.array_equal(o[k], outs[0][k]), (kernel, k)
    finally:
        gpu.set_tuning()
