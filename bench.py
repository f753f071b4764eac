"""Throughput of the WCSPH step on one MI355X.

One step = cell hash + stable radix sort + reorder (cell list), the pair
interaction (continuity, momentum with Tait pressure and Monaghan viscosity),
the device-side adaptive time step and the Verlet update.  The headline
workload is the largest single-GPU dam break: the tank with the obstacle at
dp = 0.0025 m (5,798,336 particles: 4,608,000 fluid + 1,190,336 dynamic
boundary), mixed precision (FP32 pair arithmetic on cell + offset positions,
FP64 integration), FP64 global diagnostics every 100 steps inside the timed
steps.  Inputs are resident in HBM before the timed region.

Prints one JSON line: particle-steps/s of the mixed step, the FP64 step on the
same workload for the ratio, the interaction kernel's roofline (achieved
algorithmic FP32 FLOP/s over HIP-event kernel time, and the HBM bytes per
launch from the committed counter summary), the same pair for the dam break at
dp = 0.01 m, the batched ensemble of 64 dam breaks and the paper's
artificial-viscosity study as a batch (throughput, sort/reorder HBM bandwidth
against peak), the steps and calls around the step (symplectic scheme, gate
release, loads on solids, MPS operators) and the FP64 CPU oracle timed on
this host.
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FLOPs per interacting ordered pair (FMA = 2, sqrt/rcp = 1 each):
# fluid i with fluid j, fluid i with boundary j (no delta term), boundary i
# with fluid j (continuity only)
FLOP_FF, FLOP_FB, FLOP_BF = 50, 44, 24
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32, dual-issue (packed) figure
PEAK_FP32_SCALAR_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
HBM_TBS = 8.0


#: counter summary of the headline workload's interaction kernel
PROFILE = os.path.join(ROOT, "profiles", "k_interact_mixed_dambreak_obstacle_dp0.0025.txt")
KERNEL_SOURCES = ("paper_2306_01959_amd/csrc/interact.hip", "paper_2306_01959_amd/csrc/update.h",
                  "paper_2306_01959_amd/csrc/common.h")


def kernel_name(shape, precision="Mixed"):
    """Name of the interaction kernel launched for an autotuner shape
    ((kernel, split, group), or (split, group) for the row-split kernel)."""
    shape = tuple(shape)
    if len(shape) == 2:
        shape = (1,) + shape
    shape = shape[:3]          # the XCD run does not change the kernel
    if shape[0] == 2:
        return "k_interact_g<%s, %d, false, false>" % (precision, shape[2])
    if shape[0] in (3, 4):
        return "k_interact_c<%s, %d, false, false, %s>" % (
            precision, 8 if shape[2] == 8 else 16, "true" if shape[0] == 4 else "false")
    return "k_interact<%s, %d, %d, false, false>" % (precision, shape[1], shape[2])


def measured_traffic(kernel, profile=PROFILE):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel's), or None when the
    summary is for another kernel or the kernel's sources changed since."""
    import hashlib
    try:
        kv = {}
        with open(profile) as f:
            for ln in f:
                if " = " in ln:
                    k, v = ln.split(" = ", 1)
                    kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in KERNEL_SOURCES:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    if kv.get("source_sha256") != h.hexdigest() or kv.get("kernel") != kernel:
        return None
    return float(kv["traffic_bytes_per_launch"])


def hip_runtime():
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    return C.CDLL("libamdhip64.so.7")


class Events:
    """hipEvent_t pairs around one region (by default the interaction kernel)
    of every `every`-th step (NULL for the other steps)."""

    def __init__(self, hip, n, every=1, start=0):
        self.hip = hip
        self.n = n
        self.steps = list(range(start, n, every))
        self.begin = (C.c_void_p * n)()
        self.end = (C.c_void_p * n)()
        for arr in (self.begin, self.end):
            for k in self.steps:
                h = C.c_void_p()
                assert hip.hipEventCreate(C.byref(h)) == 0
                arr[k] = h
        hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]

    def mean_ms(self):
        return self.mean_ms_upto(self.n)

    def mean_ms_upto(self, m):
        """Mean over the sampled steps below m (the steps a shorter run used)."""
        tot = 0.0
        ms = C.c_float()
        steps = [k for k in self.steps if k < m]
        for k in steps:
            rc = self.hip.hipEventElapsedTime(C.byref(ms), self.begin[k], self.end[k])
            assert rc == 0, f"hipEventElapsedTime of step {k}: error {rc}"
            tot += ms.value
        return tot / len(steps)

    def close(self):
        for arr in (self.begin, self.end):
            for k in self.steps:
                self.hip.hipEventDestroy(C.c_void_p(arr[k]))


EVENT_EVERY = 10   # interaction kernels timed with HIP events: every 10th step


REPEATS = 5  # timed segments; the step time reported is their median


def time_gpu(scene_obj, precision, steps, warmup, hip, repeats=REPEATS, diag_every=0,
             probes=None):
    """`warmup` untimed steps, then `steps` steps in `repeats` consecutive
    segments, each bracketed by events on the library's stream (device
    time); the interaction kernel is timed by events inside the library every
    EVENT_EVERY-th step.  diag_every > 0: diagnostics (with `probes`) after
    every step index that is a multiple of it, inside the timed segments (the
    cell list they build is the next step's)."""
    import torch
    from paper_2306_01959_amd import lib
    sim = lib.Simulation(scene_obj, precision)
    sim.run(warmup, -1.0, 0)
    d0, _ = sim.diagnostics()
    repeats = max(1, min(repeats, steps))
    lens = [steps // repeats + (1 if r < steps % repeats else 0) for r in range(repeats)]
    ev = Events(hip, max(lens), every=EVENT_EVERY)
    seg_ms, kern = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = warmup
    nd = 0
    for seg in lens:  # exactly `steps` steps in all
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        k = 0
        while k < seg:
            m = seg - k
            if diag_every > 0:
                m = min(m, diag_every - step % diag_every)
            sub = [(C.c_void_p * m).from_address(C.addressof(arr) + k * C.sizeof(C.c_void_p))
                   for arr in (ev.begin, ev.end)]
            sim.run_profiled(m, -1.0, step, sub[0], sub[1])
            step += m
            k += m
            if diag_every > 0 and step % diag_every == 0:
                sim.diagnostics(probes)
                nd += 1
        b.record()
        b.synchronize()
        seg_ms.append(a.elapsed_time(b) / seg)
        kern.append(ev.mean_ms_upto(seg))
    t1 = time.perf_counter()
    d1, _ = sim.diagnostics()
    ev.close()
    pairs = [(d1[k] - d0[k]) / steps for k in ("pairs_ff", "pairs_fb", "pairs_bf")]
    flop = FLOP_FF * pairs[0] + FLOP_FB * pairs[1] + FLOP_BF * pairs[2]
    assert d1["n_nonfinite"] == 0, "non-finite state"
    return dict(wall_s=t1 - t0, steps=steps, diagnostics=nd, ms_per_step=float(np.median(seg_ms)),
                segment_ms=seg_ms, interact_ms=float(np.median(kern)), pairs_per_step=pairs,
                flop_per_launch=flop, sim_time=d1["time"] - d0["time"], umax=d1["umax"],
                x_front=d1["x_front"])


def config_table(hip, steps_scale=1.0):
    """Both precisions on configurations 1, 2, 3 and 5 (the dam break at dp
    0.02, 0.01, and with the obstacle at 0.005 and 0.0025 m), each in its
    autotuned launch shape."""
    from paper_2306_01959_amd import autotune, scene
    rows = []
    # diagnostics cadence of the workloads: configuration 3 reads four probes
    # (x = 0.84 - dp, y = 0.3, z = 0.02 ... 0.14) every 10 steps,
    # configuration 5 the global diagnostics every 100 steps
    cadence = {3: (10, [[0.84 - 0.005, 0.3, z] for z in (0.02, 0.06, 0.10, 0.14)]),
               5: (100, None)}
    for cfg, steps in ((1, 400), (2, 400), (3, 200), (5, 100)):
        sc = scene.config_scene(cfg)
        every, probes = cadence.get(cfg, (0, None))
        for prec in ("mixed", "fp64"):
            shape = autotune.tune(sc, prec)
            r = time_gpu(sc, prec, max(REPEATS, int(steps * steps_scale)), 20, hip,
                         diag_every=every, probes=probes)
            pps = sc.n / (r["ms_per_step"] * 1e-3)
            rows.append({
                "config": cfg, "precision": prec, "particles": sc.n, "fluid": sc.n_fluid,
                "shape": list(shape), "ms_per_step": r["ms_per_step"],
                "particle_steps_per_s": pps,
                "fluid_particle_steps_per_s": sc.n_fluid / (r["ms_per_step"] * 1e-3),
                "pairs_per_s": sum(r["pairs_per_step"]) / (r["ms_per_step"] * 1e-3),
                "interact_ms": r["interact_ms"],
                "interact_tflops": r["flop_per_launch"] / (r["interact_ms"] * 1e-3) / 1e12,
                "diagnostics_every": every, "diagnostics_in_timed_steps": r["diagnostics"],
            })
            print(json.dumps(rows[-1]), flush=True)
    return rows


# Algorithmic HBM bytes of the cell list per particle-step: 16 (the key
# written, read by the histogram, read again with the permutation written in
# one stable counting pass) + twice the resident state (gathered and written:
# x, y, z, u, u at t - dt as FP64, 72 B; rho - rho0 at both levels as FP32,
# 8 B; the id, 4 B) + 4 B per cell of the cell table.
ALG_KEY_BYTES = 16
STATE_BYTES = {"mixed": 84, "fp64": 92}
CELL_TABLE_BYTES = 4
# The bytes this design moves (design overhead over the algorithmic ones):
SORT_BYTES_FIRST = 44   # pass 0: histogram reads x, y, z, id and writes the key; scatter
                        # reads the key, writes key + index
SORT_BYTES_FIRST_COUNTED = 12  # pass 0 when the previous (fused row-split) step wrote
                               # the keys and counted their digits: scatter only
SORT_BYTES_FIRST_KEYS = 16  # pass 0 when the previous (fused) step wrote the keys:
                            # histogram reads the key; scatter as above
SORT_BYTES_PASS = 20    # later passes: + the index read
REORDER_BYTES = 4 + 4 + 84 + 84 + 40  # perm + key in, state gathered (84 B) and written,
                                      # interaction view written (40 B)
REORDER_BYTES_WALL = 4 + 4 + 16  # a fixed wall's particle left in place (mixed): key
                                 # and density in, the view's density part out (the
                                 # update wrote both levels to the destination)
TABLE_BYTES = 4 + 4 + 4  # per cell-table entry (same launch as the reorder): its previous
                         # value read as the search hint, one key probed, the entry written


def time_ensemble(steps, hip, n_inst=64, seed=4, graph=True, retune=False, scenes=None,
                  workload=None):
    """The batched ensemble: n_inst dam breaks with dp drawn from {0.02,
    0.015, 0.01} m and alpha from U[0, 0.1] (or the given scenes), mixed
    precision, lagged-dt fused interaction + update, replayed 40-step HIP
    graphs."""
    import torch
    from paper_2306_01959_amd import lib, scene
    if scenes is None:
        scenes = scene.ensemble(n_inst, master_seed=seed)
    n_inst = len(scenes)
    from paper_2306_01959_amd import autotune
    ens = lib.Ensemble(scenes, "mixed", stream=torch.cuda.Stream())
    period = 40
    steps = max(period, (steps + period - 1) // period * period)
    mode = lib.RUN_LAGGED
    # the table's launch shape from the first step on (else tuned on the
    # warmed-up batch)
    shape = None if retune else autotune.cached_ensemble_shape(ens, "mixed")
    ens.run(period, -1.0, 0, mode)                      # eager warm-up, steps 0..39
    if shape is None:
        shape = autotune.tune_ensemble(ens, "mixed", use_cache=not retune, verbose=retune)
    # restart from the scenes so the timed steps follow the warm-up directly
    ens = lib.Ensemble(scenes, "mixed", stream=ens.stream)
    ens.run(period, -1.0, 0, mode)
    d0 = ens.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(steps, -1.0, period, mode | (lib.RUN_GRAPH if graph else 0))  # graph replays
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = ens.diagnostics()
    step = period + steps
    # kernel times of the same steps, eager with events (sampled)
    kern = {}
    for name, region in (("sort", lib.REGION_SORT), ("reorder", lib.REGION_REORDER),
                         ("interact", lib.REGION_INTERACT), ("step", lib.REGION_STEP)):
        # one whole refresh period of steady-state steps: a call's first two
        # steps gather every particle (the fixed walls stay in place from
        # the third on, as in the graph replays), so the period sampled is
        # steps 2 .. period + 1 of the call
        ev = Events(hip, period + 2, start=2)
        ens.run_profiled(period + 2, -1.0, step, ev.begin, ev.end, region=region, mode=mode)
        torch.cuda.synchronize()
        kern[name] = ev.mean_ms()
        ev.close()
        step += period + 2
    assert all(d["n_nonfinite"] == 0 for d in d1), "non-finite state"
    n = ens.n
    # sort key: 2 x (cells) keys of the cell list plus 2 sub-cell bits; the
    # sub-cell bits are sorted only once per graph period, the passes below
    # are those of the other steps
    key_bits = int(np.ceil(np.log2(2 * sum(int(np.prod(s.params["dims"])) for s in scenes)))) + 2
    passes = max(1, (key_bits - 2 + 7) // 8)
    # the fused interaction writes the next sort's keys when its occupancy is
    # fixed (mixed: wave per group, or row split with groups of 16 or more);
    # the sampled steps follow a fused step
    keys_written = shape[0] == 2 or (shape[0] == 1 and shape[2] >= 16)
    counted = shape[0] == 1 and shape[2] >= 16   # the row-split kernel also counts
    first = (SORT_BYTES_FIRST_COUNTED if counted else
             SORT_BYTES_FIRST_KEYS if keys_written else SORT_BYTES_FIRST)
    sort_bytes = n * (first + SORT_BYTES_PASS * (passes - 1))
    cells = sum(int(np.prod(s.params["dims"])) for s in scenes)
    n_wall = sum(int(s.is_boundary.sum()) for s in scenes)
    reorder_bytes = ((n - n_wall) * REORDER_BYTES + n_wall * REORDER_BYTES_WALL
                     + (2 * cells + 1) * TABLE_BYTES)
    alg_bytes = n * (ALG_KEY_BYTES + 2 * STATE_BYTES["mixed"]) + CELL_TABLE_BYTES * cells
    pairs = [(d1[0][k] - d0[0][k]) / steps for k in ("pairs_ff", "pairs_fb", "pairs_bf")]
    flop = FLOP_FF * pairs[0] + FLOP_FB * pairs[1] + FLOP_BF * pairs[2]

    def bw(nbytes, ms):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"achieved": gbs, "peak": HBM_TBS * 1e3, "unit": "GB/s",
                "frac": gbs / (HBM_TBS * 1e3), "kernel_ms": ms, "bytes_per_launch": nbytes}

    counts = [s.n for s in scenes]
    return {
        "value": n * steps / (t1 - t0),
        "unit": "particle-steps/s",
        "ms_per_step": (t1 - t0) / steps * 1e3,
        "steps": steps,
        "workload": (workload or f"{n_inst} dam-break instances (same tank), dp from "
                     "{0.02, 0.015, 0.01} m, alpha ~ U[0, 0.1]") +
                    ", mixed FP32, lagged CFL dt per instance, fused interaction + update, "
                    + ("40-step HIP graph replays" if graph else "eager launches"),
        "instances": n_inst,
        "interaction_shape": list(shape),
        "particles": n,
        "particles_per_instance": {"min": min(counts), "max": max(counts)},
        # the sort and reorder together against the algorithmic bytes
        "sort_reorder": dict(
            bw(alg_bytes, kern["sort"] + kern["reorder"]),
            bytes_model="16 B key + 2 x 84 B state per particle + 4 B per cell",
            design_bytes_per_launch=sort_bytes + reorder_bytes,
            design_over_algorithmic=(sort_bytes + reorder_bytes) / alg_bytes),
        # each launch sequence against the bytes this design moves
        "sort": dict(bw(sort_bytes, kern["sort"]), passes=passes, key_bits=key_bits,
                     bytes_model="design bytes",
                     first_pass_keys=("written and counted by the fused update" if counted
                                      else "written by the fused update") if keys_written
                     else "computed from the positions"),
        "reorder": dict(bw(reorder_bytes, kern["reorder"]), bytes_model="design bytes",
                        wall_particles=n_wall,
                        walls="left in place (steady state: a call's steps 2 on)"),
        "interact": {"kernel_ms": kern["interact"], "achieved": flop / (kern["interact"] * 1e-3)
                     / 1e12, "unit": "TFLOP/s", "peak": PEAK_FP32_TFLOPS,
                     "flop_per_launch": flop},
        "eager_step_ms": kern["step"],
        "pairs_per_step": sum(pairs),
        "pairs_per_s": sum(pairs) * steps / (t1 - t0),
    }




def time_alpha_study(steps, hip, retune=False, graph=True, dp=0.005):
    """The paper's artificial-viscosity study as one batch: the obstacle dam
    break at dp = 0.005 m once per alpha0 in {0.1, 0.01, 0.001, 0.0001}, with
    the paper's 2h = 3 l0 and c0 = 20 sqrt(g H_W)."""
    from paper_2306_01959_amd import scene
    scenes = scene.alpha_study(dp)
    r = time_ensemble(steps, hip, scenes=scenes, retune=retune, graph=graph,
                      workload=f"{len(scenes)} obstacle dam breaks at dp={dp:g} m, one per "
                               "alpha0 in {0.1, 0.01, 0.001, 0.0001}, 2h = 3 l0, "
                               "c0 = 20 sqrt(g 0.3)")
    r["instances_by_name"] = [s.name for s in scenes]
    r["nu0"] = [scene.viscosity_label(s.params) for s in scenes]
    return r


# Algorithmic FP64 work of one explicit MPS neighbour pair with a field
# (eqs. mpsw, mpspnd, mpsgrad, mpslap, mpssigmai2; FMA = 2, sqrt / division =
# 1): displacement 3, r^2 5, weight 3, density 1, centroid sums 6, field
# difference 1, Laplacian sum 2, gradient sums 12.
FLOP_MPS = 33
PEAK_FP64_TFLOPS = 78.6


def _event_ms(fn, calls):
    """Mean device time of `calls` calls of fn() between two events on the
    current stream (the library's)."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(calls):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / calls


def time_extras(sc, verlet_ms, steps=40, warmup=5, calls=20):
    """What the library computes around the step, each on the headline
    workload unless stated: the two-stage symplectic scheme (two
    interactions per step), the gate-release dam break at dp = 0.005 m (a
    moving boundary, the paper's Verlet scheme), the loads (force on the
    obstacle's upstream face and on every wall particle, probe pressures and
    their impulse), and the explicit MPS operators (r_e = 2.1 dp, cells of
    edge r_e)."""
    import torch
    from paper_2306_01959_amd import lib, scene
    dp = sc.params["dp"]
    out = {}
    # two-stage symplectic scheme, device-side dt
    sim = lib.Simulation(sc, "mixed", scheme=lib.SCHEME_SYMPLECTIC)
    sim.run(warmup, -1.0, 0)
    ms = _event_ms(lambda: sim.run(steps, -1.0, warmup), 1) / steps
    d, _ = sim.diagnostics()
    assert d["n_nonfinite"] == 0, "non-finite state"
    out["symplectic"] = {
        "workload": "headline workload, two-stage symplectic predictor-corrector (two "
                    "interactions and cell lists per step), mixed, device-side dt",
        "steps": steps, "ms_per_step": ms, "value": sc.n / (ms * 1e-3),
        "unit": "particle-steps/s", "over_verlet_step": ms / verlet_ms}
    # loads at that state: the force sums and the probes synchronise the stream
    face = (0.84, 0.84 + 2 * dp, 0.24, 0.36, 0.0, 0.16)
    walls = (-10.0, 10.0, -10.0, 10.0, -10.0, 10.0)
    probes = [[0.84 - dp, 0.3, z] for z in (0.02, 0.06, 0.10, 0.14)]
    nf, _, _ = sim.neighbour_stats()
    wall_pairs = int(nf[sc.is_boundary].sum())
    loads = {"workload": "headline workload after the symplectic steps; host-synchronous calls"}
    for name, box in (("face_force", face), ("wall_force", walls)):
        f, cnt = sim.boundary_force(box)
        t0 = time.perf_counter()
        for _ in range(calls):
            sim.boundary_force(box)
        us = (time.perf_counter() - t0) / calls * 1e6
        loads[name] = {"us_per_call": us, "boundary_particles": cnt, "force_N": list(f)}
    loads["wall_force"]["fluid_pairs"] = wall_pairs
    loads["wall_force"]["pairs_per_s"] = wall_pairs / (loads["wall_force"]["us_per_call"] * 1e-6)
    sim.probe_impulse(probes, reset=True)
    t0 = time.perf_counter()
    for _ in range(calls):
        sim.probe_impulse(probes)
    loads["probe_impulse"] = {"us_per_call": (time.perf_counter() - t0) / calls * 1e6,
                              "probes": len(probes)}
    out["loads"] = loads
    del sim
    torch.cuda.empty_cache()
    # moving boundary: the gate release, the paper's Verlet scheme
    gate = scene.gate_release(0.005, 7)
    sim = lib.Simulation(gate, "mixed")
    sim.run(warmup, -1.0, 0)
    ms = _event_ms(lambda: sim.run(steps, -1.0, warmup), 1) / steps
    out["gate_release"] = {
        "workload": "gate-release dam break at dp = 0.005 m, gate lifted at 1.25 m/s, "
                    "Verlet scheme, mixed, device-side dt",
        "particles": gate.n, "steps": steps, "ms_per_step": ms,
        "value": gate.n / (ms * 1e-3), "unit": "particle-steps/s"}
    del sim
    torch.cuda.empty_cache()
    # explicit MPS operators on the headline particle set
    re = 2.1 * dp
    lo = [min(v.min(), 0.0) - 0.05 for v in (sc.x, sc.y, sc.z)]
    hi = [max(v.max(), 0.0) + 0.05 for v in (sc.x, sc.y, sc.z)]
    msc = sc.copy()
    msc.params = scene.make_params(dp, h_factor=re / (2 * dp), lo=lo, hi=hi)
    sim = lib.Simulation(msc, "fp64")
    sim.build_cells()
    nf, nb, _ = sim.neighbour_stats()   # the same set: r^2 < (2h)^2 = r_e^2
    pairs = int(nf.sum() + nb.sum())
    n0, lam = lib.mps_constants(dp, re)
    m = lib.SphMps(re, n0, lam, 0.98, 0.2, dp)
    f64 = dict(dtype=torch.float64, device="cuda")
    phi = torch.rand(sc.n, **f64)
    pnd, lap, sig = (torch.empty(sc.n, **f64) for _ in range(3))
    grad = torch.empty(3 * sc.n, **f64)
    surf = torch.empty(sc.n, dtype=torch.int32, device="cuda")

    def mps():
        lib.check(sim.lib.sph_mps_operators(
            C.byref(sim.params), C.byref(sim.state), sim.ws_ptr, C.byref(m), phi.data_ptr(),
            pnd.data_ptr(), lap.data_ptr(), grad.data_ptr(), sig.data_ptr(), surf.data_ptr(),
            sim._s()))
    mps()
    ms = _event_ms(mps, calls)
    achieved = FLOP_MPS * pairs / (ms * 1e-3) / 1e12
    out["mps_operators"] = {
        "workload": "headline particle set, r_e = 2.1 dp, cells of edge r_e, FP64: particle "
                    "number density, Laplacian and gradient of a field, centroid deviation, "
                    "free-surface flags",
        "ms_per_call": ms, "particles": sc.n, "neighbour_pairs": pairs,
        "pairs_per_s": pairs / (ms * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "flop_model": f"{FLOP_MPS} FP64 per neighbour pair"}}
    del sim
    torch.cuda.empty_cache()
    return out


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_window(scene_obj, threads, seconds, warm=1, max_steps=2000):
    """The FP64 oracle on this host: `warm` steps, then single steps of the
    same workload until `seconds` elapse (at least 3); particle-steps/s.
    threads: OpenMP threads (None: the OpenMP default, which follows
    OMP_NUM_THREADS, i.e. this host's share of cores)."""
    from oracle import orc
    orc.build(force=False)
    if threads:
        orc.set_threads(threads)
    used = orc.max_threads()
    p = orc.par(scene_obj.params)
    st = orc.State(scene_obj)
    orc.run(p, st, warm, dt_mode=1)
    k = 0
    t0 = time.perf_counter()
    while True:
        orc.run(p, st, 1, dt_mode=1)
        k += 1
        el = time.perf_counter() - t0
        if (el >= seconds and k >= 3) or k >= max_steps:
            break
    return dict(value=scene_obj.n * k / el, threads=used, steps=k, warm=warm, seconds=el)


def cpu_baseline(sc_head, sc_small, seconds_all=12.0, seconds_one=8.0):
    """The FP64 C oracle, untuned, on this host's cores: a window of the
    headline workload with every hardware thread, and the dp = 0.01 m dam
    break on one thread."""
    head = oracle_window(sc_head, None, seconds_all)
    one = oracle_window(sc_small, 1, seconds_one)
    model = cpu_model()
    return {
        "value": head["value"], "unit": "particle-steps/s", "cores": head["threads"],
        "kind": "oracle",
        "sample": f"{head['steps']} steps of the headline workload ({sc_head.n} particles) "
                  f"after {head['warm']} warm-up step, FP64 C oracle (OpenMP over particles, "
                  f"{head['threads']} threads), {head['seconds']:.1f} s; CPU {model}",
        "cpu_model": model,
        "one_thread": {"value": one["value"], "unit": "particle-steps/s", "cores": 1,
                       "sample": f"{one['steps']} steps of the dp = 0.01 m dam break "
                                 f"({sc_small.n} particles) after {one['warm']} warm-up step, "
                                 f"{one['seconds']:.1f} s"},
    }


def headline_workload(sc):
    return ("3D dam break with obstacle: tank 1.6x0.6x0.6 m, water 0.4x0.6x0.3 m, box "
            "0.12x0.12x0.16 m at x=0.9 m, dp=0.0025 m, h=1.2*sqrt(3)*dp, Wendland C2, "
            "alpha=0.01, delta=0.1, CFL 0.2 (device-side adaptive dt), full sort every step, "
            "FP64 diagnostics every 100 steps; mixed FP32 interaction + FP64 integration")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison")
    ap.add_argument("--retune", action="store_true", help="ignore the autotune table")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-small", action="store_true", help="skip the dp = 0.01 m dam break")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the batched ensemble (profiling its kernels alone)")
    ap.add_argument("--ensemble-eager", action="store_true",
                    help="ensemble without HIP graphs (for counter collection)")
    ap.add_argument("--ensemble-steps", type=int, default=200,
                    help="timed ensemble steps (rounded up to whole 40-step graphs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--configs", action="store_true",
                    help="only the per-configuration table (configs 1, 2, 3, 5; both precisions)")
    ap.add_argument("--small-only", action="store_true",
                    help="only the dp = 0.01 m dam break, mixed (profiling its kernels alone)")
    ap.add_argument("--no-alpha", action="store_true", help="skip the alpha-study batch")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the symplectic, gate-release, loads and MPS legs")
    ap.add_argument("--alpha-only", action="store_true",
                    help="only the alpha-study batch (profiling its kernels alone)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_01959_amd import autotune, scene
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hip = hip_runtime()

    if args.calib_copy:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE of this kernel
        # calibrate the same counters read on the interaction kernel
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.configs:
        config_table(hip)
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble": time_ensemble(args.ensemble_steps, hip,
                                                    graph=not args.ensemble_eager,
                                                    retune=args.retune)}), flush=True)
        return
    if args.alpha_only:
        print(json.dumps({"alpha_study": time_alpha_study(args.ensemble_steps, hip,
                                                          retune=args.retune,
                                                          graph=not args.ensemble_eager)}),
              flush=True)
        return
    sc2 = scene.config_scene(2)
    if args.small_only:
        autotune.tune(sc2, "mixed", use_cache=not args.retune)
        r = time_gpu(sc2, "mixed", args.steps, args.warmup, hip)
        print(json.dumps({"small_mixed_ms_per_step": r["ms_per_step"],
                          "interact_ms": r["interact_ms"]}), flush=True)
        return

    # headline: the dam break with the obstacle at dp = 0.0025 m, diagnostics
    # every 100 steps (FP64 mass, momentum, energy) inside the timed steps
    sc = scene.config_scene(5)
    shapes = {"mixed": autotune.tune(sc, "mixed", use_cache=not args.retune,
                                     verbose=args.retune)}
    mixed = time_gpu(sc, "mixed", args.steps, args.warmup, hip, diag_every=100)
    print(f"# headline mixed: {mixed['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        shapes["fp64"] = autotune.tune(sc, "fp64", use_cache=not args.retune,
                                       verbose=args.retune)
        fp64 = time_gpu(sc, "fp64", args.steps, args.warmup, hip, diag_every=100)
        print(f"# headline fp64: {fp64['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    value = sc.n / (mixed["ms_per_step"] * 1e-3)
    achieved = mixed["flop_per_launch"] / (mixed["interact_ms"] * 1e-3) / 1e12
    kname = kernel_name(shapes["mixed"])
    out = {
        "metric": "particle-steps/s of WCSPH step, mixed-FP32 vs FP64 on 1 GPU, + ensemble batch",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": mixed["steps"],
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "timing": f"median over {len(mixed['segment_ms'])} consecutive segments of the "
                  f"{mixed['steps']} timed steps (events on the library's stream)",
        "fluid_particle_steps_per_s": sc.n_fluid / (mixed["ms_per_step"] * 1e-3),
        "pairs_per_s": sum(mixed["pairs_per_step"]) / (mixed["ms_per_step"] * 1e-3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": headline_workload(sc),
            "particles": sc.n, "fluid": sc.n_fluid, "boundary": sc.n_boundary,
            "precision": "mixed", "parallelism": "single GPU",
            "diagnostics_in_timed_steps": mixed["diagnostics"],
            "interaction_shape": {k: list(v) for k, v in shapes.items()},
        },
        "roofline": {
            "kernel": kname,
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(kname),
            "kernel_ms": mixed["interact_ms"],
            "flop_per_launch": mixed["flop_per_launch"],
            "flop_model": f"{FLOP_FF} per fluid-fluid, {FLOP_FB} per fluid-boundary, "
                          f"{FLOP_BF} per boundary-fluid interacting ordered pair",
            "pairs_per_launch": {"ff": mixed["pairs_per_step"][0],
                                 "fb": mixed["pairs_per_step"][1],
                                 "bf": mixed["pairs_per_step"][2]},
            "frac_of_scalar_issue_peak": achieved / PEAK_FP32_SCALAR_TFLOPS,
        },
    }
    if fp64 is not None:
        v64 = sc.n / (fp64["ms_per_step"] * 1e-3)
        out["fp64"] = {"value": v64, "ms_per_step": fp64["ms_per_step"],
                       "interact_ms": fp64["interact_ms"],
                       "kernel": kernel_name(shapes["fp64"], "Fp64")}
        out["mixed_over_fp64"] = value / v64
    if not args.no_small:
        small = {"workload": "3D dam break, same tank without the obstacle, dp=0.01 m, "
                             "hydrostatic start", "particles": sc2.n}
        for prec in ("mixed",) + (() if args.no_fp64 else ("fp64",)):
            shp = autotune.tune(sc2, prec, use_cache=not args.retune)
            r = time_gpu(sc2, prec, max(REPEATS, 2 * args.steps), args.warmup, hip)
            small[prec] = {"value": sc2.n / (r["ms_per_step"] * 1e-3),
                           "ms_per_step": r["ms_per_step"], "interact_ms": r["interact_ms"],
                           "interact_tflops": r["flop_per_launch"] / (r["interact_ms"] * 1e-3)
                           / 1e12, "shape": list(shp)}
        if "fp64" in small:
            small["mixed_over_fp64"] = small["mixed"]["value"] / small["fp64"]["value"]
        out["dambreak_dp0.01"] = small
    if not args.no_ensemble:
        out["ensemble"] = time_ensemble(args.ensemble_steps, hip, retune=args.retune)
    if not args.no_alpha:
        out["alpha_study"] = time_alpha_study(args.ensemble_steps, hip, retune=args.retune)
    if not args.no_extras:
        out["extras"] = time_extras(sc, mixed["ms_per_step"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc, sc2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
