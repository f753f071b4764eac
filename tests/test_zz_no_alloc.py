"""sph_run_noalloc (the library's static scratch instead of a caller
workspace) against sph_run on a fresh workspace, through the C ABI.

Both run the same kernels in the same launch shapes on the same inputs, so
the states must agree bit for bit (stricter than the parity tolerances
against the oracle: FP64 1e-12, mixed 1e-5 relative L2).  Two calls in a row, the
second on a smaller system, so the second call runs on scratch the first
one filled."""
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
    return lib


def _compare(gpu, sc, precision, nsteps):
    ref = gpu.Simulation(sc, precision)
    ref.run(nsteps, -1.0, 0)
    want = ref.fetch()
    d_ref, _ = ref.diagnostics()
    sim = gpu.Simulation(sc, precision)
    sim.run_noalloc(nsteps, -1.0, 0)
    got = sim.fetch()
    for k in want:
        assert np.array_equal(got[k], want[k]), (precision, sc.n, k)
        den = max(np.linalg.norm(want[k]), 1e-300)
        assert np.linalg.norm(got[k] - want[k]) / den <= 1e-12
    # the state really moved
    assert not np.array_equal(want["z"], sc.z)
    return d_ref


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_equals_run_twice(gpu, precision):
    big = scene.config_scene(1)                                   # 28,392 particles
    small = scene.dam_break(0.03, 11, alpha=0.05, name="small")  # fewer particles
    assert small.n < big.n
    print(f"noalloc {precision}: n={big.n} then n={small.n}", flush=True)
    _compare(gpu, big, precision, 25)
    _compare(gpu, small, precision, 12)


def test_noalloc_rejects_oversize(gpu):
    import ctypes as C
    sc = scene.config_scene(1)
    p = gpu.make_params(sc.params, "fp64")
    need = C.c_size_t(0)
    gpu.check(gpu.load().sph_workspace_bytes(C.byref(p), 4_000_000, C.byref(need)))
    assert need.value > (32 << 20)
    sim = gpu.Simulation(sc, "fp64")
    st = gpu.SphState()
    C.memmove(C.addressof(st), C.addressof(sim.state), C.sizeof(st))
    st.n = 4_000_000                                   # validated before any launch
    rc = gpu.load().sph_run_noalloc(C.byref(p), C.byref(st), 1, -1.0, 0, None)
    assert rc == gpu.SPH_E_SIZE
    assert b"static scratch" in gpu.load().sph_last_error()
