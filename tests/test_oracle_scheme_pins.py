"""Pins of the oracle's two-stage symplectic scheme and of moving boundary
particles (a gate lifted at constant speed).

* Constant acceleration is integrated exactly (free fall), and a boundary
  particle with a prescribed velocity moves exactly with it, in both the
  paper's Verlet scheme and the symplectic one.
* The symplectic scheme is second-order accurate: on an interacting cloud the
  error of r, u and rho falls by about 4 when dt halves (a plausible slip,
  such as the corrector kicking with the rates at t, or the position taking
  u at t only, makes it first order).
* Without body force and walls the total momentum is conserved to rounding.
* A wall moving into resting fluid compresses it: both densities rise.
"""
import numpy as np
import pytest

from paper_2306_01959_amd import scene


def _cloud(n, seed, **kw):
    return scene.random_cloud(n, seed, dp=0.01, box=0.06, **kw)


def test_symplectic_free_fall_and_moving_wall_exact(oracle_lib):
    orc = oracle_lib
    prm = scene.make_params(0.01, lo=(-0.1, -0.1, -0.1), hi=(0.5, 0.5, 0.6))
    s = scene.random_cloud(2, 0, dp=0.01)
    s.params = prm
    s.x[:] = [0.1, 0.3]
    s.y[:] = [0.2, 0.2]
    s.z[:] = [0.3, 0.1]
    s.ux[:] = [0.7, 0.0]
    s.uy[:] = [-0.2, 0.0]
    s.uz[:] = [1.5, 1.25]          # particle 1: a gate particle moving up
    s.is_boundary[:] = [False, True]
    p = orc.par(prm)
    dt, nsteps = 1e-3, 130
    for scheme in ("symplectic", "verlet"):
        st = orc.State(s)
        if scheme == "symplectic":
            orc.run_symplectic(p, st, nsteps, dt_mode=0, dt_in=np.full(nsteps, dt))
        else:
            orc.run(p, st, nsteps, dt_mode=0, dt_in=np.full(nsteps, dt))
        t = nsteps * dt
        assert st.x[0] == pytest.approx(0.1 + 0.7 * t, rel=1e-12)
        assert st.z[0] == pytest.approx(0.3 + 1.5 * t - 0.5 * 9.81 * t * t, rel=1e-12)
        assert st.uz[0] == pytest.approx(1.5 - 9.81 * t, rel=1e-12)
        assert st.z[1] == pytest.approx(0.1 + 1.25 * t, rel=1e-12)
        assert st.x[1] == 0.3 and st.uz[1] == 1.25


def _run(orc, s, scheme, dt, T):
    p = orc.par(s.params)
    st = orc.State(s)
    n = int(round(T / dt))
    if scheme == "symplectic":
        orc.run_symplectic(p, st, n, dt_mode=0, dt_in=np.full(n, dt))
    else:
        orc.run(p, st, n, dt_mode=0, dt_in=np.full(n, dt))
    return np.concatenate([st.x, st.y, st.z]), np.concatenate([st.ux, st.uy, st.uz]), st.rho


def test_symplectic_second_order(oracle_lib):
    """Errors against a dt/16 reference at T = 4 ms: halving dt divides them
    by about 4 (between 3.3 and 4.8) for positions, velocities and densities."""
    orc = oracle_lib
    s = _cloud(400, 3, speed=0.3, drho=3.0, alpha=0.05)
    T, dt0 = 4e-3, 2e-4
    ref = _run(orc, s, "symplectic", dt0 / 16, T)
    errs = []
    for dt in (dt0, dt0 / 2, dt0 / 4):
        got = _run(orc, s, "symplectic", dt, T)
        errs.append([np.abs(g - r).max() for g, r in zip(got, ref)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.3) and np.all(ratios < 4.8), ratios


def test_symplectic_conserves_momentum(oracle_lib):
    """No body force and no walls: both kicks apply antisymmetric pair forces
    to every particle with the same dt, so the total momentum stays at its
    initial value to rounding over 200 steps at the CFL time step."""
    orc = oracle_lib
    s = _cloud(500, 7, speed=0.5, drho=4.0, alpha=0.05, gravity=(0, 0, 0))
    p = orc.par(s.params)
    st = orc.State(s)
    d0 = orc.diagnostics(p, st)
    orc.run_symplectic(p, st, 200, dt_mode=1)
    d = orc.diagnostics(p, st)
    scale = s.params["mass"] * np.abs(s.ux).sum()
    for k in ("px", "py", "pz"):
        assert abs(d[k] - d0[k]) <= 1e-12 * scale, k
    assert d["e_kin"] != pytest.approx(d0["e_kin"], rel=1e-2)   # the cloud did interact


def test_moving_wall_compresses(oracle_lib):
    """A boundary particle moving towards a resting fluid particle: the
    relative velocity closes the pair, so both densities rise (eq. sphrho,
    first term), and the fluid particle is pushed away by the viscous term."""
    orc = oracle_lib
    prm = scene.make_params(0.01, lo=(-0.1,) * 3, hi=(0.3,) * 3, alpha=0.1,
                            gravity=(0, 0, 0))
    p = orc.par(prm)
    h = prm["h"]
    x = np.array([0.1, 0.1])
    y = np.array([0.1, 0.1])
    z = np.array([0.1, 0.1 + h])
    uz = np.array([1.25, 0.0])          # wall below, moving up into the fluid
    zero = np.zeros(2)
    ax, ay, az, dr, mm = orc.rates(p, x, y, z, zero, zero, uz, np.full(2, 1000.0),
                                   np.array([True, False]))
    assert dr[0] > 0 and dr[1] > 0
    assert az[1] > 0 and az[0] == 0.0
