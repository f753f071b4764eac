"""ctypes wrapper around the FP64 C oracle (test infrastructure only).

The oracle works on particles in their original order; every function takes
and returns numpy float64 arrays.  The C source cites the equations of the
paper that each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle: plain C, FP64, no FMA contraction, OpenMP."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcPar(C.Structure):
    _fields_ = [
        ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
        ("gamma", C.c_double), ("alpha", C.c_double), ("delta", C.c_double),
        ("mass", C.c_double), ("eta2_coef", C.c_double), ("cfl", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
        ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
        ("cs", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("c_const", C.c_int32), ("delta_all", C.c_int32),
        ("verlet_ns", C.c_int32),
    ]


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(OrcPar)
        L.orc_kernel_w.restype = C.c_double
        L.orc_kernel_w.argtypes = [C.c_double, C.c_double]
        L.orc_kernel_f.restype = C.c_double
        L.orc_kernel_f.argtypes = [C.c_double, C.c_double]
        L.orc_pressure.restype = C.c_double
        L.orc_pressure.argtypes = [P, C.c_double]
        L.orc_sound.restype = C.c_double
        L.orc_sound.argtypes = [P, C.c_double]
        L.orc_internal_energy.restype = C.c_double
        L.orc_internal_energy.argtypes = [P, C.c_double]
        L.orc_cells.restype = C.c_int
        L.orc_cells.argtypes = [P, C.c_int64, _D, _D, _D, _I32, _I32, _I32,
                                _I64, _I64]
        L.orc_neighbours.restype = C.c_int64
        L.orc_neighbours.argtypes = [P, C.c_int64, _D, _D, _D, _I64, _I64,
                                     C.c_int64]
        L.orc_rates.restype = C.c_int
        L.orc_rates.argtypes = [P, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _U8,
                                _D, _D, _D, _D, _D, _I64]
        L.orc_dt_cfl.restype = C.c_double
        L.orc_dt_cfl.argtypes = [P, C.c_int64, _D, _D, _D, _D, _U8]
        L.orc_update.restype = None
        L.orc_update.argtypes = [P, C.c_int64, C.c_int, C.c_double] + [_D] * 11 \
            + [_D] * 4 + [_U8]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_int64] + [_D] * 11 + [_U8, C.c_int64,
                                                         C.c_int64, C.c_int,
                                                         _D, _D, _D]
        L.orc_run_symplectic.restype = C.c_int
        L.orc_run_symplectic.argtypes = [P, C.c_int64] + [_D] * 11 + [_U8, C.c_int64, C.c_int,
                                                                    _D, _D]
        L.orc_diagnostics.restype = C.c_int
        L.orc_diagnostics.argtypes = [P, C.c_int64, _D, _D, _D, _D, _D, _D,
                                      _D, _U8, _D]
        L.orc_probes.restype = None
        L.orc_probes.argtypes = [P, C.c_int64, _D, _D, _D, _D, _U8, C.c_int32,
                                 _D, _D]
        L.orc_boundary_force.restype = C.c_int
        L.orc_boundary_force.argtypes = [P, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _U8,
                                         _D, _D]
        L.orc_impulse_step.restype = C.c_double
        L.orc_impulse_step.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_mps_weight.restype = C.c_double
        L.orc_mps_weight.argtypes = [C.c_double, C.c_double]
        L.orc_mps_lattice.restype = None
        L.orc_mps_lattice.argtypes = [C.c_double, C.c_double, _D, _D]
        L.orc_mps_operators.restype = C.c_int
        L.orc_mps_operators.argtypes = [P, C.c_int64, _D, _D, _D, _D] + [C.c_double] * 6 + \
            [_D, _D, _D, _D, _I32]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def par(params: Dict[str, object], *, c_const: bool = False,
        delta_all: bool = False, **override) -> OrcPar:
    p = dict(params)
    p.update(override)
    g = p["g"]
    o = p["origin"]
    d = p["dims"]
    return OrcPar(h=p["h"], rho0=p["rho0"], c0=p["c0"], gamma=p["gamma"],
                  alpha=p["alpha"], delta=p["delta"], mass=p["mass"],
                  eta2_coef=p["eta2_coef"], cfl=p["cfl"], gx=g[0], gy=g[1],
                  gz=g[2], ox=o[0], oy=o[1], oz=o[2], cs=p["cell_size"],
                  nx=d[0], ny=d[1], nz=d[2], c_const=int(c_const),
                  delta_all=int(delta_all), verlet_ns=int(p["verlet_ns"]))


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def kernel_w(q: float, h: float) -> float:
    return lib().orc_kernel_w(q, h)


def kernel_f(q: float, h: float) -> float:
    return lib().orc_kernel_f(q, h)


def pressure(p: OrcPar, rho: float) -> float:
    return lib().orc_pressure(C.byref(p), rho)


def sound(p: OrcPar, rho: float) -> float:
    return lib().orc_sound(C.byref(p), rho)


def internal_energy(p: OrcPar, rho: float) -> float:
    return lib().orc_internal_energy(C.byref(p), rho)


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def cells(p: OrcPar, x, y, z):
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    cx = np.zeros(n, np.int32)
    cy = np.zeros(n, np.int32)
    cz = np.zeros(n, np.int32)
    start = np.zeros(p.nx * p.ny * p.nz + 1, np.int64)
    order = np.zeros(n, np.int64)
    rc = lib().orc_cells(C.byref(p), n, _d(x), _d(y), _d(z),
                         cx.ctypes.data_as(_I32), cy.ctypes.data_as(_I32),
                         cz.ctypes.data_as(_I32), start.ctypes.data_as(_I64),
                         order.ctypes.data_as(_I64))
    assert rc == 0
    return cx, cy, cz, start, order


def neighbours(p: OrcPar, x, y, z, want_pairs: bool = False,
               max_pairs: int = 50_000_000):
    """Per-particle neighbour counts and optionally the (i, j) pair list."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    cnt = np.zeros(n, np.int64)
    total = lib().orc_neighbours(C.byref(p), n, _d(x), _d(y), _d(z),
                                 cnt.ctypes.data_as(_I64), None, 0)
    assert total >= 0
    if not want_pairs:
        return cnt, None
    assert total <= max_pairs
    pairs = np.zeros((max(total, 1), 2), np.int64)
    t2 = lib().orc_neighbours(C.byref(p), n, _d(x), _d(y), _d(z),
                              cnt.ctypes.data_as(_I64),
                              pairs.ctypes.data_as(_I64), total)
    assert t2 == total
    return cnt, pairs[:total]


def rates(p: OrcPar, x, y, z, ux, uy, uz, rho, is_bnd,
          want_counts: bool = False):
    """(ax, ay, az, drho, mumax) at one state; optionally the pair counts
    (fluid-fluid, fluid-boundary, boundary-fluid)."""
    arrs = [_f64(a) for a in (x, y, z, ux, uy, uz, rho)]
    b = _u8(is_bnd)
    n = arrs[0].size
    outs = [np.zeros(n) for _ in range(5)]
    cnt = np.zeros(3, np.int64)
    rc = lib().orc_rates(C.byref(p), n, *[_d(a) for a in arrs],
                         b.ctypes.data_as(_U8), *[_d(o) for o in outs],
                         cnt.ctypes.data_as(_I64))
    assert rc == 0
    if want_counts:
        return tuple(outs), tuple(int(v) for v in cnt)
    return tuple(outs)


def dt_cfl(p: OrcPar, ax, ay, az, mumax, is_bnd) -> float:
    a = [_f64(v) for v in (ax, ay, az, mumax)]
    b = _u8(is_bnd)
    return lib().orc_dt_cfl(C.byref(p), a[0].size, *[_d(v) for v in a],
                            b.ctypes.data_as(_U8))


class State:
    """Oracle state in original particle order (two Verlet levels)."""

    def __init__(self, scene):
        self.x, self.y, self.z = _f64(scene.x).copy(), _f64(scene.y).copy(), _f64(scene.z).copy()
        self.ux, self.uy, self.uz = _f64(scene.ux).copy(), _f64(scene.uy).copy(), _f64(scene.uz).copy()
        self.uxm, self.uym, self.uzm = self.ux.copy(), self.uy.copy(), self.uz.copy()
        self.rho = _f64(scene.rho).copy()
        self.rhom = self.rho.copy()
        self.is_bnd = _u8(scene.is_boundary)
        self.step = 0

    @property
    def n(self) -> int:
        return self.x.size

    def arrays(self):
        return (self.x, self.y, self.z, self.ux, self.uy, self.uz, self.uxm,
                self.uym, self.uzm, self.rho, self.rhom)


def update(p: OrcPar, st: State, euler: bool, dt: float, rates5) -> None:
    ax, ay, az, dr = [_f64(v) for v in rates5[:4]]
    lib().orc_update(C.byref(p), st.n, int(euler), float(dt),
                     *[_d(a) for a in st.arrays()], _d(ax), _d(ay), _d(az),
                     _d(dr), st.is_bnd.ctypes.data_as(_U8))


def run(p: OrcPar, st: State, nsteps: int, dt_mode: int = 1,
        dt_in: Optional[np.ndarray] = None, keep_rates: bool = False):
    """Advance `st` by nsteps; returns (dt per step, last rates or None)."""
    n = st.n
    dts = np.zeros(max(nsteps, 1))
    dti = _f64(dt_in if dt_in is not None else np.zeros(max(nsteps, 1)))
    rbuf = np.zeros(5 * n) if keep_rates else None
    rc = lib().orc_run(C.byref(p), n, *[_d(a) for a in st.arrays()],
                       st.is_bnd.ctypes.data_as(_U8), st.step, nsteps, dt_mode,
                       _d(dti), _d(dts), _d(rbuf) if rbuf is not None else None)
    assert rc == 0
    st.step += nsteps
    rates5 = tuple(rbuf.reshape(5, n)) if rbuf is not None else None
    return dts[:nsteps], rates5


def run_symplectic(p: OrcPar, st: State, nsteps: int, dt_mode: int = 1,
                   dt_in: Optional[np.ndarray] = None) -> np.ndarray:
    """Advance `st` by nsteps of the two-stage symplectic scheme; returns
    the dt of every step."""
    n = st.n
    dts = np.zeros(max(nsteps, 1))
    dti = _f64(dt_in if dt_in is not None else np.zeros(max(nsteps, 1)))
    rc = lib().orc_run_symplectic(C.byref(p), n, *[_d(a) for a in st.arrays()],
                                  st.is_bnd.ctypes.data_as(_U8), nsteps, dt_mode, _d(dti),
                                  _d(dts))
    assert rc == 0
    st.step += nsteps
    return dts[:nsteps]


def diagnostics(p: OrcPar, st: State) -> Dict[str, float]:
    out = np.zeros(11)
    rc = lib().orc_diagnostics(C.byref(p), st.n, _d(st.x), _d(st.y), _d(st.z),
                               _d(st.ux), _d(st.uy), _d(st.uz), _d(st.rho),
                               st.is_bnd.ctypes.data_as(_U8), _d(out))
    assert rc == 0
    keys = ["mass", "px", "py", "pz", "e_kin", "e_pot", "e_int", "umax",
            "x_front", "n_nonfinite", "n_outside"]
    return dict(zip(keys, out.tolist()))


def probes(p: OrcPar, st_or_arrays, pts) -> np.ndarray:
    if isinstance(st_or_arrays, State):
        st = st_or_arrays
        x, y, z, rho, isb = st.x, st.y, st.z, st.rho, st.is_bnd
    else:
        x, y, z, rho, isb = st_or_arrays
        x, y, z, rho, isb = _f64(x), _f64(y), _f64(z), _f64(rho), _u8(isb)
    pts = _f64(np.asarray(pts).reshape(-1))
    npts = pts.size // 3
    out = np.zeros(max(npts, 1))
    lib().orc_probes(C.byref(p), x.size, _d(x), _d(y), _d(z), _d(rho),
                     isb.ctypes.data_as(_U8), npts, _d(pts), _d(out))
    return out[:npts]


def boundary_force(p: OrcPar, st_or_arrays, box):
    """(force vector, particle count) of the boundary particles inside
    box = (x0, x1, y0, y1, z0, z1)."""
    if isinstance(st_or_arrays, State):
        st = st_or_arrays
        arrs = (st.x, st.y, st.z, st.ux, st.uy, st.uz, st.rho)
        isb = st.is_bnd
    else:
        *arrs, isb = st_or_arrays
        arrs = [_f64(a) for a in arrs]
        isb = _u8(isb)
    b = _f64(np.asarray(box, np.float64).reshape(6))
    out = np.zeros(4)
    rc = lib().orc_boundary_force(C.byref(p), arrs[0].size, *[_d(a) for a in arrs],
                                  isb.ctypes.data_as(_U8), _d(b), _d(out))
    assert rc == 0
    return out[:3].copy(), int(out[3])


def impulse_step(I: float, p_prev: float, p_now: float, dt: float) -> float:
    return float(lib().orc_impulse_step(float(I), float(p_prev), float(p_now), float(dt)))


def mps_weight(r: float, re: float) -> float:
    return float(lib().orc_mps_weight(float(r), float(re)))


def mps_lattice(l0: float, re: float):
    """(n0, lambda0) of the fully filled support on the cubic lattice."""
    n0 = C.c_double(0.0)
    lam = C.c_double(0.0)
    lib().orc_mps_lattice(float(l0), float(re), C.byref(n0), C.byref(lam))
    return n0.value, lam.value


def mps_operators(p: OrcPar, x, y, z, phi, re, n0, lambda0, beta1=0.98, rho1=0.2, l0=None):
    """Per particle: (pnd, laplacian of phi, gradient of phi (3, n), sigma,
    surface flag); phi may be None (laplacian and gradient are then None)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    ph = _f64(phi) if phi is not None else None
    pnd = np.zeros(n)
    lap = np.zeros(n)
    grad = np.zeros(3 * n)
    sig = np.zeros(n)
    surf = np.zeros(n, np.int32)
    rc = lib().orc_mps_operators(C.byref(p), n, _d(x), _d(y), _d(z),
                                 _d(ph) if ph is not None else None, float(re), float(n0),
                                 float(lambda0), float(beta1), float(rho1), float(l0),
                                 _d(pnd), _d(lap), _d(grad), _d(sig),
                                 surf.ctypes.data_as(_I32))
    assert rc == 0
    if ph is None:
        return pnd, None, None, sig, surf
    return pnd, lap, grad.reshape(3, n), sig, surf
