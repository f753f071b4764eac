"""Pins of the oracle's diagnostics, probe operator and lagged time step.

Each test checks one output of the oracle against a fact fixed from outside
it: hand-placed particle sets whose answer is known by construction, closed
forms on lattices, the exact constant-acceleration motion, and the
definition of the lagged time step (eq. sphdt one step late) rebuilt from the
separately pinned rates, bound and update routines.
"""
import math

import numpy as np
import pytest

from paper_2306_01959_amd import scene


def _scene(x, y, z, isb, params, ux=None, uy=None, uz=None, rho=None):
    n = len(x)
    z0 = np.zeros(n)
    return scene.Scene("pin", np.asarray(x, float).copy(), np.asarray(y, float).copy(),
                       np.asarray(z, float).copy(),
                       z0.copy() if ux is None else np.asarray(ux, float).copy(),
                       z0.copy() if uy is None else np.asarray(uy, float).copy(),
                       z0.copy() if uz is None else np.asarray(uz, float).copy(),
                       np.full(n, float(params["rho0"])) if rho is None
                       else np.asarray(rho, float).copy(),
                       np.asarray(isb, bool).copy(), dict(params))


def _box_params(**kw):
    return scene.make_params(0.02, lo=(0.0, 0.0, 0.0), hi=(1.0, 0.4, 0.4), **kw)


# ------------------------------------------------------------- surge front

def test_front_hand_placed(oracle_lib):
    """x_front = max x over fluid particles that have a fluid particle within
    2h.  Built by hand: a fluid pair (included), a lone fluid particle far
    ahead (spray, excluded), and a fluid particle further ahead whose only
    neighbour is a boundary particle (excluded)."""
    orc = oracle_lib
    prm = _box_params()
    h = prm["h"]
    x = [0.30, 0.30 + 1.5 * h,       # fluid pair, 1.5h apart: front = 0.30 + 1.5h
         0.70,                       # isolated fluid particle
         0.85, 0.85 + 0.5 * h]       # fluid particle + boundary particle beside it
    y = [0.2] * 5
    z = [0.2] * 5
    isb = [False, False, False, False, True]
    st = orc.State(_scene(x, y, z, isb, prm))
    d = orc.diagnostics(orc.par(prm), st)
    assert d["x_front"] == 0.30 + 1.5 * h
    # the pair pulled apart to exactly 2h (outside the strict support): no
    # fluid particle has a fluid neighbour, the front is -inf
    x2 = list(x)
    x2[1] = 0.30 + 2.0 * h
    st2 = orc.State(_scene(x2, y, z, isb, prm))
    assert orc.diagnostics(orc.par(prm), st2)["x_front"] == -math.inf
    # a second fluid particle beside the one near the boundary makes both count
    x3 = x + [0.85 - 0.5 * h]
    st3 = orc.State(_scene(x3, y + [0.2], z + [0.2], isb + [False], prm))
    assert orc.diagnostics(orc.par(prm), st3)["x_front"] == 0.85


def test_front_across_cells(oracle_lib):
    """The front neighbour test sees fluid neighbours in adjacent cells: a
    pair straddling a cell face at 1.9h apart diagonally counts."""
    orc = oracle_lib
    prm = _box_params()
    h, cs, o = prm["h"], prm["cell_size"], prm["origin"]
    face = o[0] + 5 * cs
    d = 1.9 * h / math.sqrt(3.0)
    x = [face - 0.5 * d, face + 0.5 * d]
    y = [0.2 - 0.5 * d, 0.2 + 0.5 * d]
    z = [0.2 - 0.5 * d, 0.2 + 0.5 * d]
    st = orc.State(_scene(x, y, z, [False, False], prm))
    assert orc.diagnostics(orc.par(prm), st)["x_front"] == x[1]


# ------------------------------------------------ momentum and energies

def _lattice(nx, ny, nz, dp, corner):
    ax = [corner[k] + (np.arange(n) + 0.5) * dp for k, n in enumerate((nx, ny, nz))]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return xx.ravel(), yy.ravel(), zz.ravel()


def test_momentum_energy_translated_lattice(oracle_lib):
    """A lattice translating at U: momentum = M_f U, kinetic energy = M_f |U|^2 / 2,
    potential energy -sum m g.r = m g sum z with the lattice's sum of z in
    closed form; boundary particles count for the mass only."""
    orc = oracle_lib
    prm = _box_params()
    dp, m = prm["dp"], prm["mass"]
    nx, ny, nz = 6, 5, 4
    x, y, z = _lattice(nx, ny, nz, dp, (0.1, 0.1, 0.1))
    nf = x.size
    bx, by, bz = _lattice(3, 3, 1, dp, (0.6, 0.1, 0.05))
    U = np.array([0.7, -0.3, 0.25])
    n = nf + bx.size
    isb = np.r_[np.zeros(nf, bool), np.ones(bx.size, bool)]
    ux = np.r_[np.full(nf, U[0]), np.zeros(bx.size)]
    uy = np.r_[np.full(nf, U[1]), np.zeros(bx.size)]
    uz = np.r_[np.full(nf, U[2]), np.zeros(bx.size)]
    st = orc.State(_scene(np.r_[x, bx], np.r_[y, by], np.r_[z, bz], isb, prm, ux, uy, uz))
    d = orc.diagnostics(orc.par(prm), st)
    M = nf * m
    assert d["mass"] == pytest.approx(n * m, rel=1e-15)
    assert d["px"] == pytest.approx(M * U[0], rel=1e-13)
    assert d["py"] == pytest.approx(M * U[1], rel=1e-13)
    assert d["pz"] == pytest.approx(M * U[2], rel=1e-13)
    assert d["e_kin"] == pytest.approx(0.5 * M * float(U @ U), rel=1e-13)
    # sum of z over the fluid lattice: nx ny sum_k (0.1 + (k + 1/2) dp)
    sum_z = nx * ny * sum(0.1 + (k + 0.5) * dp for k in range(nz))
    assert d["e_pot"] == pytest.approx(m * 9.81 * sum_z, rel=1e-13)
    # a potential raised by a rigid lift of dz is m g dz per fluid particle
    st.z[:nf] += 0.05
    d2 = orc.diagnostics(orc.par(prm), st)
    assert d2["e_pot"] - d["e_pot"] == pytest.approx(M * 9.81 * 0.05, rel=1e-10)
    assert d["umax"] == pytest.approx(float(np.sqrt(U @ U)), rel=1e-15)
    # internal energy at rho0 is zero; a uniform density gives M_all e(rho)
    assert abs(d["e_int"]) < 1e-12 * M * 9.81
    st.rho[:] = 1004.0
    d3 = orc.diagnostics(orc.par(prm), st)
    assert d3["e_int"] == pytest.approx(n * m * orc.internal_energy(orc.par(prm), 1004.0),
                                        rel=1e-12)


def test_free_fall_cloud_momentum_and_energy(oracle_lib):
    """Particles more than 2h apart do not interact, so every one falls
    freely (a = g exactly): after time t the fluid momentum equals
    sum m (u0 + g t), and E_kin + E_pot is constant to rounding under the
    exact constant-acceleration update, through Euler and Verlet steps."""
    orc = oracle_lib
    prm = scene.make_params(0.02, lo=(-1.0, -1.0, -3.0), hi=(2.0, 2.0, 2.0))
    h = prm["h"]
    rng = np.random.default_rng(3)
    k = np.arange(5)
    gx, gy, gz = np.meshgrid(k, k, k, indexing="ij")
    sp = 3.0 * h
    x = gx.ravel() * sp + 0.1
    y = gy.ravel() * sp + 0.1
    z = gz.ravel() * sp + 0.5
    n = x.size
    u = rng.uniform(-0.5, 0.5, size=(3, n))
    st = orc.State(_scene(x, y, z, np.zeros(n, bool), prm, *u))
    p = orc.par(prm)
    d0 = orc.diagnostics(p, st)
    dt = 2.5e-4
    nsteps = 90                       # two Euler resets inside
    orc.run(p, st, nsteps, dt_mode=0, dt_in=np.full(nsteps, dt))
    t = nsteps * dt
    d1 = orc.diagnostics(p, st)
    m = prm["mass"]
    assert d1["px"] == pytest.approx(m * u[0].sum(), rel=1e-12, abs=1e-15)
    assert d1["py"] == pytest.approx(m * u[1].sum(), rel=1e-12, abs=1e-15)
    assert d1["pz"] == pytest.approx(m * (u[2].sum() - n * 9.81 * t), rel=1e-12)
    e0 = d0["e_kin"] + d0["e_pot"]
    e1 = d1["e_kin"] + d1["e_pot"]
    assert abs(e1 - e0) <= 1e-12 * (abs(d0["e_pot"]) + d0["e_kin"])
    assert d1["e_kin"] != pytest.approx(d0["e_kin"], rel=1e-3)  # energy moved


# ------------------------------------------------------ outside / non-finite

def test_outside_and_nonfinite_counts(oracle_lib):
    """Particles beyond the grid on each side are counted once each; every
    non-finite value among x, y, z, u, rho counts once."""
    orc = oracle_lib
    prm = _box_params()
    o = np.asarray(prm["origin"])
    top = o + np.asarray(prm["dims"]) * prm["cell_size"]
    base = np.array([0.5, 0.2, 0.2])
    pts = [base + [0.01 * k, 0, 0] for k in range(4)]
    outside = []
    for ax in range(3):
        lo = base.copy()
        lo[ax] = o[ax] - 0.01
        hi = base.copy()
        hi[ax] = top[ax] + 0.01
        outside += [lo, hi]
    pts = np.array(pts + outside)
    n = len(pts)
    st = orc.State(_scene(pts[:, 0], pts[:, 1], pts[:, 2], np.zeros(n, bool), prm))
    d = orc.diagnostics(orc.par(prm), st)
    assert d["n_outside"] == 6 and d["n_nonfinite"] == 0
    st.ux[0] = np.nan
    st.uz[1] = np.inf
    st.rho[2] = np.nan
    st.y[3] = -np.inf                 # also outside (binned to cell 0)
    d2 = orc.diagnostics(orc.par(prm), st)
    assert d2["n_nonfinite"] == 4
    assert d2["n_outside"] == 7


# ------------------------------------------------------------- probes (eq. sphpa)

def test_probe_shepard_operator(oracle_lib):
    """Shepard average (eq. sphpa): a uniform fluid pressure is returned
    exactly; a pressure linear in x, probed at the centre of a symmetric
    lattice, returns the centre value (odd terms cancel); boundary particles
    never contribute; a probe with no fluid within 2h reads 0."""
    orc = oracle_lib
    prm = scene.make_params(0.01, lo=(-0.05,) * 3, hi=(0.3,) * 3)
    p = orc.par(prm)
    dp = prm["dp"]
    x, y, z = _lattice(12, 12, 12, dp, (0.0, 0.0, 0.0))
    n = x.size
    B = prm["rho0"] * prm["c0"] ** 2 / prm["gamma"]

    def rho_of(P):
        return prm["rho0"] * (1.0 + P / B) ** (1.0 / prm["gamma"])

    centre = np.array([[6 * dp, 6 * dp, 6 * dp]])
    isb = np.zeros(n, bool)
    rho = np.full(n, rho_of(1500.0))
    got = orc.probes(p, (x, y, z, rho, isb), centre)
    assert got[0] == pytest.approx(orc.pressure(p, rho[0]), rel=1e-13)
    # linear in x about the centre (the lattice is symmetric about it)
    P = 800.0 + 3.0e4 * (x - centre[0, 0])
    rho_lin = rho_of(P)
    got = orc.probes(p, (x, y, z, rho_lin, isb), centre)
    P_back = np.array([orc.pressure(p, r) for r in rho_lin])
    w = np.abs(P_back - P).max()
    assert got[0] == pytest.approx(800.0, abs=1e-9 * 3.0e4 + 10 * w)
    # boundary particles are ignored: mark the x > centre half as boundary
    # with a wild density; the fluid half alone, uniform, gives its own value
    isb2 = x > centre[0, 0]
    rho2 = np.where(isb2, rho_of(9.0e4), rho_of(1500.0))
    got = orc.probes(p, (x, y, z, rho2, isb2), centre)
    assert got[0] == pytest.approx(orc.pressure(p, rho_of(1500.0)), rel=1e-12)
    # a dry probe
    far = np.array([[0.25, 0.25, 0.25]])
    assert orc.probes(p, (x, y, z, rho, isb), far)[0] == 0.0


# ------------------------------------------------------------- lagged dt

def test_lagged_dt_is_previous_bound(oracle_lib):
    """dt_mode 2: step 0 takes its own bound, step k > 0 the bound of step
    k - 1 (eq. sphdt one step late).  Rebuilt here from the rates, bound and
    update routines, step by step from saved states, and the resulting
    states agree bit for bit."""
    orc = oracle_lib
    s = scene.config_scene(1)
    p = orc.par(s.params)
    warm = orc.State(s)
    orc.run(p, warm, 30, dt_mode=1)       # a developed state (flow under way)
    lag_state = orc.State(s)
    ref_state = orc.State(s)
    for dst in (lag_state, ref_state):
        for a, b in zip(dst.arrays(), warm.arrays()):
            a[:] = b
        dst.step = warm.step
    nsteps = 6
    dts, _ = orc.run(p, lag_state, nsteps, dt_mode=2)
    prev_bound = None
    for k in range(nsteps):
        st = ref_state
        r = orc.rates(p, st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho, st.is_bnd)
        bound = orc.dt_cfl(p, r[0], r[1], r[2], r[4], st.is_bnd)
        dt = bound if k == 0 else prev_bound
        assert dts[k] == dt, k
        step = st.step
        orc.update(p, st, step % 40 == 0, dt, r)
        st.step += 1
        prev_bound = bound
    assert len(set(dts.tolist())) > 1          # the bound really changes
    for a, b in zip(lag_state.arrays(), ref_state.arrays()):
        assert np.array_equal(a, b)


# ---------------------------------------------------- hydrostatics, delta = 0.1

@pytest.mark.slow
def test_hydrostatic_column_with_delta_drift_bound(oracle_lib):
    """With the paper's delta = 0.1 (delta term over fluid pairs only) the
    resting column drifts from rho0 g (H - z): about 4-5 % of rho0 g H at the
    floor after 0.6 s.  Held to a 6 % bound (and above 1 %, so the drift is
    real) so that the documented behaviour cannot change silently."""
    orc = oracle_lib
    s = scene.resting_column(0.02, 0, tank=(0.2, 0.2, 0.4), H=0.3, alpha=0.1,
                             delta=0.1)
    p = orc.par(s.params)
    st = orc.State(s)
    h, c0, H = s.params["h"], s.params["c0"], 0.3
    dt = s.params["cfl"] * h / c0
    orc.run(p, st, int(0.6 / dt), dt_mode=1)
    zs = np.array([2 * h + 0.001, 0.1, 0.15, 0.2, H - 2 * h])
    pts = np.array([[0.1, 0.1, zz] for zz in zs])
    pr = orc.probes(p, st, pts)
    err = (pr - 1000.0 * 9.81 * (H - zs)) / (1000.0 * 9.81 * H)
    assert 0.01 < np.abs(err).max() < 0.06, err
