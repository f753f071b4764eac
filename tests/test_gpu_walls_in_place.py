"""The fixed-wall shortcut on the GPU, through the C ABI.

From the third step of a call, and outside the two steps from each refresh,
while no boundary particle moves, the boundary particles keep their sorted
positions (all of an instance's walls follow all of its fluid in key order,
and their keys do not change), so a step's gather leaves them in place and
only copies their densities and rewrites their view.  That must give the same
run bit for bit as gathering every particle (sph_tuning.full_gather = 1): the
same order, positions, velocities and densities, in both precisions; for
single systems, from a call that starts between refreshes, across a refresh;
for batches, lagged fused steps and graph replays, a 4.5 M-particle ensemble;
and with a moving gate, which the update detects, so every step gathers every
particle.
"""
import numpy as np
import pytest

from paper_2306_01959_amd import scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_01959_amd import lib
    lib.load()
    yield lib
    lib.set_tuning()


def _both(gpu, make, advance):
    """(ids, fetched state) of the same run with every particle gathered and
    with the shortcut."""
    out = []
    for full in (1, 0):
        gpu.set_tuning(full_gather=full)
        obj = make()
        advance(obj)
        out.append((obj.ids(), obj.fetch()))
    gpu.set_tuning()
    return out


def _assert_same(label, a, b):
    (ia, ra), (ib, rb) = a, b
    assert np.array_equal(ia, ib), label
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), (label, k)
    print(f"\n{label}: identical ({ia.size} particles)", flush=True)


@pytest.mark.parametrize("precision, cfg, nsteps, step0", [
    ("mixed", 2, 45, 0),    # refresh at step 40 inside the call
    ("fp64", 1, 50, 5),     # starts between refreshes: the walls' first refresh at 40
    ("mixed", 3, 24, 30),   # obstacle: more wall than water near the block
])
def test_single_system_same_bits(gpu, precision, cfg, nsteps, step0):
    sc = scene.config_scene(cfg)
    a, b = _both(gpu, lambda: gpu.Simulation(sc, precision),
                 lambda s: s.run(nsteps, -1.0, step0))
    _assert_same(f"configuration {cfg} {precision}, steps {step0}..{step0 + nsteps - 1}", a, b)


@pytest.mark.parametrize("mode", ["lagged+graph", "plain"])
def test_batch_same_bits(gpu, mode):
    """Eight uneven instances: lagged fused steps with 40-step graph replays
    (130 steps), or plain steps (45)."""
    import torch
    scenes = scene.ensemble(8, master_seed=21, dps=(0.03, 0.04, 0.05))
    flags = gpu.RUN_LAGGED | gpu.RUN_GRAPH if mode != "plain" else 0
    n = 130 if mode != "plain" else 45
    # graphs are captured on a stream of the caller's (not the null stream)
    a, b = _both(gpu, lambda: gpu.Ensemble(scenes, "mixed", stream=torch.cuda.Stream()),
                 lambda e: e.run(n, -1.0, 0, mode=flags))
    _assert_same(f"8-instance batch, {mode}, {n} steps", a, b)


def test_large_ensemble_same_bits(gpu):
    """The 64-instance ensemble (4.5 M particles), lagged fused steps across
    a refresh."""
    scenes = scene.ensemble()
    a, b = _both(gpu, lambda: gpu.Ensemble(scenes, "mixed"),
                 lambda e: e.run(44, -1.0, 0, mode=gpu.RUN_LAGGED))
    _assert_same("64-instance ensemble, lagged, 44 steps", a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_moving_gate_gathers_everything(gpu, precision):
    """The gate's particles move: the first update raises the flag, so no
    step takes the shortcut; the run equals the full gather and the gate
    has moved."""
    s = scene.gate_release(0.02, 7)
    a, b = _both(gpu, lambda: gpu.Simulation(s, precision), lambda m: m.run(30, -1.0, 0))
    _assert_same(f"gate release {precision}, 30 steps", a, b)
    gate = s.is_boundary & (np.abs(s.uz) > 0)
    assert gate.any() and np.all(b[1]["z"][gate] > s.z[gate])
