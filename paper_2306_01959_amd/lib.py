"""ctypes binding of libwcsph.so (the C ABI in include/wcsph.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (tensors) and the stream.  The library must be
built (python -m paper_2306_01959_amd.build); importing this module on a
machine without it, or calling into it without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libwcsph.so")

SPH_OK, SPH_E_INVAL, SPH_E_HIP, SPH_E_RANGE, SPH_E_STATE, SPH_E_SIZE = 0, -1, -2, -3, -4, -5
SPH_FP64, SPH_MIXED = 0, 1
SPH_C_TAIT, SPH_C_CONST = 0, 1
SPH_DELTA_FLUID, SPH_DELTA_ALL = 0, 1
SCHEME_VERLET, SCHEME_SYMPLECTIC = 0, 1
FLAG_NONFINITE, FLAG_OUTSIDE, FLAG_DENSITY, FLAG_DT_CFL = 1, 2, 4, 8
BOUNDARY_BIT = np.uint32(1 << 31)

REGION_INTERACT, REGION_SORT, REGION_REORDER, REGION_STEP = 0, 1, 2, 3
RUN_LAGGED, RUN_GRAPH = 1, 2
MAX_INSTANCES = 4096

#: every symbol include/wcsph.h declares
EXPORTS = ("sph_version", "sph_last_error", "sph_check_params", "sph_set_tuning",
           "sph_get_split", "sph_workspace_bytes",
           "sph_workspace_init", "sph_set_density", "sph_get_density", "sph_build_cells",
           "sph_interact", "sph_neighbour_stats", "sph_step", "sph_run", "sph_run_noalloc",
           "sph_run_profiled",
           "sph_diagnostics", "sph_boundary_force", "sph_probe_impulse",
           "sph_mps_constants", "sph_mps_operators",
           "sph_batch_workspace_bytes", "sph_batch_workspace_init",
           "sph_batch_set_density", "sph_batch_get_density", "sph_batch_build_cells",
           "sph_batch_interact", "sph_batch_run", "sph_batch_run_profiled",
           "sph_batch_diagnostics")


class SphParams(C.Structure):
    _fields_ = [
        ("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
        ("gamma", C.c_double), ("alpha", C.c_double), ("delta", C.c_double),
        ("g", C.c_double * 3), ("eta2_coef", C.c_double), ("cfl", C.c_double),
        ("mass", C.c_double), ("origin", C.c_double * 3), ("cell_size", C.c_double),
        ("dims", C.c_int32 * 3), ("verlet_ns", C.c_int32), ("precision", C.c_int32),
        ("c_mode", C.c_int32), ("delta_pairs", C.c_int32), ("scheme", C.c_int32),
    ]


_P = C.c_void_p


SPH_KERNEL_AUTO, SPH_KERNEL_ROWS, SPH_KERNEL_GROUPS, SPH_KERNEL_COOP, SPH_KERNEL_COOP2 = (
    0, 1, 2, 3, 4)


class SphTuning(C.Structure):
    _fields_ = [("split_fp64", C.c_int32), ("split_mixed", C.c_int32),
                ("group_fp64", C.c_int32), ("group_mixed", C.c_int32),
                ("kernel_fp64", C.c_int32), ("kernel_mixed", C.c_int32),
                ("xcd_run_fp64", C.c_int32), ("xcd_run_mixed", C.c_int32),
                ("full_gather", C.c_int32)]


class SphState(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _P) for k in (
        "x", "y", "z", "ux", "uy", "uz", "uxm", "uym", "uzm", "rho", "rhom", "id",
        "x_alt", "y_alt", "z_alt", "ux_alt", "uy_alt", "uz_alt", "uxm_alt", "uym_alt",
        "uzm_alt", "rho_alt", "rhom_alt", "id_alt")] + [
        ("cells_valid", C.c_int32), ("reserved", C.c_int32)]


class SphDiag(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("mom", C.c_double * 3), ("e_kin", C.c_double),
        ("e_pot", C.c_double), ("e_int", C.c_double), ("umax", C.c_double),
        ("x_front", C.c_double), ("dt_cfl", C.c_double), ("dt_last", C.c_double),
        ("time", C.c_double), ("n", C.c_int64), ("n_fluid", C.c_int64),
        ("n_outside", C.c_int64), ("n_nonfinite", C.c_int64), ("steps", C.c_int64),
        ("pairs_ff", C.c_int64), ("pairs_fb", C.c_int64), ("pairs_bf", C.c_int64),
        ("flags", C.c_uint32), ("reserved", C.c_uint32),
    ]

    def as_dict(self) -> Dict[str, object]:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("mom", "reserved")}
        d["mom"] = tuple(self.mom)
        return d


class SphMps(C.Structure):
    _fields_ = [("re", C.c_double), ("n0", C.c_double), ("lambda0", C.c_double),
                ("beta1", C.c_double), ("rho1", C.c_double), ("l0", C.c_double)]


def mps_constants(l0: float, re: float):
    """(n0, lambda0) of the full support on the cubic lattice (eq. mpslambda)."""
    n0 = C.c_double(0.0)
    lam = C.c_double(0.0)
    check(load().sph_mps_constants(float(l0), float(re), C.byref(n0), C.byref(lam)))
    return n0.value, lam.value


class SphBatch(C.Structure):
    _fields_ = [("ninst", C.c_int32), ("reserved", C.c_int32),
                ("params", C.POINTER(SphParams)), ("counts", C.POINTER(C.c_int64))]


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libwcsph error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libwcsph.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2306_01959_amd.build")
    # torch first: the library then binds to the HIP runtime torch already
    # loaded (same soname), so both share one runtime and one device context
    import torch  # noqa: F401
    L = C.CDLL(path)
    PP, PS, PD = C.POINTER(SphParams), C.POINTER(SphState), C.POINTER(SphDiag)
    L.sph_version.restype = C.c_int
    L.sph_last_error.restype = C.c_char_p
    L.sph_check_params.argtypes = [PP]
    L.sph_set_tuning.argtypes = [C.POINTER(SphTuning)]
    L.sph_get_split.argtypes = [PP, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32)]
    L.sph_workspace_bytes.argtypes = [PP, C.c_int64, C.POINTER(C.c_size_t)]
    L.sph_workspace_init.argtypes = [PP, C.c_int64, _P, C.c_size_t, _P]
    L.sph_set_density.argtypes = [PP, PS, _P, C.c_int32, _P]
    L.sph_get_density.argtypes = [PP, PS, _P, C.c_int32, _P]
    L.sph_build_cells.argtypes = [PP, PS, _P, _P]
    L.sph_interact.argtypes = [PP, PS, _P, _P, _P, _P, _P, _P, _P]
    L.sph_neighbour_stats.argtypes = [PP, PS, _P, _P, _P, _P, _P]
    L.sph_step.argtypes = [PP, PS, _P, C.c_double, C.c_int64, _P]
    L.sph_run.argtypes = [PP, PS, _P, C.c_int64, C.c_double, C.c_int64, _P]
    L.sph_run_noalloc.argtypes = [PP, PS, C.c_int64, C.c_double, C.c_int64, _P]
    L.sph_run_profiled.argtypes = [PP, PS, _P, C.c_int64, C.c_double, C.c_int64, C.c_int32,
                                   _P, _P, _P]
    L.sph_diagnostics.argtypes = [PP, PS, _P, _P, C.c_int32, PD, _P, _P]
    L.sph_boundary_force.argtypes = [PP, PS, _P, _P, _P, _P, _P]
    L.sph_probe_impulse.argtypes = [PP, PS, _P, _P, C.c_int32, C.c_int32, _P, _P, _P]
    L.sph_mps_constants.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
    L.sph_mps_operators.argtypes = [PP, PS, _P, C.POINTER(SphMps), _P, _P, _P, _P, _P, _P,
                                    _P]
    PB = C.POINTER(SphBatch)
    L.sph_batch_workspace_bytes.argtypes = [PB, C.POINTER(C.c_size_t)]
    L.sph_batch_workspace_init.argtypes = [PB, _P, C.c_size_t, _P]
    L.sph_batch_set_density.argtypes = [PB, PS, _P, _P, C.c_int32, _P]
    L.sph_batch_get_density.argtypes = [PB, PS, _P, _P, C.c_int32, _P]
    L.sph_batch_build_cells.argtypes = [PB, PS, _P, _P]
    L.sph_batch_interact.argtypes = [PB, PS, _P, _P, _P, _P, _P, _P, _P]
    L.sph_batch_run.argtypes = [PB, PS, _P, C.c_int64, C.c_double, C.c_int64, C.c_int32, _P]
    L.sph_batch_run_profiled.argtypes = [PB, PS, _P, C.c_int64, C.c_double, C.c_int64,
                                         C.c_int32, C.c_int32, _P, _P, _P]
    L.sph_batch_diagnostics.argtypes = [PB, PS, _P, PD, _P]
    for name in EXPORTS[2:]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != SPH_OK:
        raise SphError(rc, load().sph_last_error().decode())


def set_tuning(split_fp64: int = 0, split_mixed: int = 0, group_fp64: int = 0,
               group_mixed: int = 0, kernel_fp64: int = 0, kernel_mixed: int = 0,
               xcd_run_fp64: int = 0, xcd_run_mixed: int = 0, full_gather: int = 0) -> None:
    """Process-wide interaction launch shape (0 = the library's choice);
    full_gather = 1: every step sorts and gathers every particle (the same
    results as the default, which leaves fixed walls in place)."""
    t = SphTuning()
    t.full_gather = int(full_gather)
    t.xcd_run_fp64 = int(xcd_run_fp64)
    t.xcd_run_mixed = int(xcd_run_mixed)
    t.split_fp64 = int(split_fp64)
    t.split_mixed = int(split_mixed)
    t.group_fp64 = int(group_fp64)
    t.group_mixed = int(group_mixed)
    t.kernel_fp64 = int(kernel_fp64)
    t.kernel_mixed = int(kernel_mixed)
    check(load().sph_set_tuning(C.byref(t)))


def get_split(params: "SphParams", n: int):
    """(waves per chunk, targets per group, kernel) the library will launch."""
    v = C.c_int32(0)
    g = C.c_int32(0)
    k = C.c_int32(0)
    check(load().sph_get_split(C.byref(params), int(n), C.byref(v), C.byref(g), C.byref(k)))
    return int(v.value), int(g.value), int(k.value)


def make_params(prm: Dict[str, object], precision: str = "mixed", *,
                c_mode: int = SPH_C_TAIT, delta_pairs: int = SPH_DELTA_FLUID,
                scheme: int = SCHEME_VERLET) -> SphParams:
    p = SphParams()
    for k in ("dp", "h", "rho0", "c0", "gamma", "alpha", "delta", "eta2_coef", "cfl", "mass"):
        setattr(p, k, float(prm[k]))
    p.g[:] = [float(v) for v in prm["g"]]
    p.origin[:] = [float(v) for v in prm["origin"]]
    p.cell_size = float(prm["cell_size"])
    p.dims[:] = [int(v) for v in prm["dims"]]
    p.verlet_ns = int(prm["verlet_ns"])
    p.precision = SPH_MIXED if precision == "mixed" else SPH_FP64
    p.c_mode = c_mode
    p.delta_pairs = delta_pairs
    p.scheme = int(scheme)
    return p


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class _System:
    """Device state (two copies of every array: the library ping-pongs
    between them), workspace and stream of one system or one batch."""

    def _alloc(self, n: int, precision: str, device: str, stream, ws_bytes: int) -> None:
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.precision = precision
        self.n = n
        self.stream = stream
        f64 = dict(dtype=torch.float64, device=self.dev)
        rdt = torch.float32 if precision == "mixed" else torch.float64
        self._buf = {}
        for k in ("x", "y", "z", "ux", "uy", "uz", "uxm", "uym", "uzm"):
            for suffix in ("", "_alt"):
                self._buf[k + suffix] = torch.zeros(n, **f64)
        for k in ("rho", "rhom"):
            for suffix in ("", "_alt"):
                self._buf[k + suffix] = torch.zeros(n, dtype=rdt, device=self.dev)
        for suffix in ("", "_alt"):
            self._buf["id" + suffix] = torch.zeros(n, dtype=torch.int32, device=self.dev)
        self.ws_bytes = int(ws_bytes)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        st = SphState()
        st.n = n
        for name, t in self._buf.items():
            setattr(st, name, t.data_ptr())
        st.cells_valid = 0
        st.reserved = 0
        self.state = st

    # -- plumbing ---------------------------------------------------------
    def _s(self):
        return _stream_ptr(self.stream)

    def _cur(self, name: str):
        """Tensor currently behind state field `name`."""
        ptr = getattr(self.state, name)
        for t in self._buf.values():
            if t.data_ptr() == ptr:
                return t
        raise KeyError(name)

    def _upload_arrays(self, vals, ids, rho, rhom) -> None:
        torch = self.torch
        for k, v in vals.items():
            self._cur(k).copy_(torch.from_numpy(np.ascontiguousarray(v, np.float64)))
        self._cur("id").copy_(torch.from_numpy(ids.view(np.int32)))
        dens = [torch.from_numpy(np.ascontiguousarray(r, np.float64)).to(self.dev)
                for r in (rho, rhom)]
        self.sync()  # the copies ran on torch's stream, the library may use another
        for which, t in enumerate(dens):
            self._set_density(t.data_ptr(), which)
        self.sync()
        self.state.cells_valid = 0

    def sync(self) -> None:
        self.torch.cuda.synchronize(self.dev)

    # -- read-back ----------------------------------------------------------
    def ids(self) -> np.ndarray:
        """Original index of every particle, in the current (cell) order;
        synchronises the device first (the library may run on another stream
        than torch's, whose copy would not wait for it)."""
        self.sync()
        raw = self._cur("id").cpu().numpy().view(np.uint32)
        return (raw & np.uint32(0x7FFFFFFF)).astype(np.int64)

    def density(self, which: int = 0):
        """FP64 densities (current order); synchronises the device, since the
        library may run on another stream than torch's."""
        out = self.torch.empty(self.n, dtype=self.torch.float64, device=self.dev)
        self._get_density(out.data_ptr(), which)
        self.sync()
        return out

    def fetch(self) -> Dict[str, np.ndarray]:
        """All state arrays in original particle order (numpy, FP64)."""
        self.sync()
        ids = self.ids()
        inv = np.empty_like(ids)
        inv[ids] = np.arange(ids.size)
        out = {}
        for k in ("x", "y", "z", "ux", "uy", "uz", "uxm", "uym", "uzm"):
            out[k] = self._cur(k).cpu().numpy()[inv]
        out["rho"] = self.density(0).cpu().numpy()[inv]
        out["rhom"] = self.density(1).cpu().numpy()[inv]
        return out

    def interact(self, want_mumax: bool = True):
        """Rates at the current state, FP64 tensors in current (cell) order."""
        torch = self.torch
        if not self.state.cells_valid:
            self.build_cells()
        outs = [torch.empty(self.n, dtype=torch.float64, device=self.dev) for _ in range(5)]
        self._interact([o.data_ptr() for o in outs[:4]],
                       outs[4].data_ptr() if want_mumax else None)
        return outs

    def rates_by_id(self):
        """(ax, ay, az, drho, mumax) in original particle order."""
        outs = self.interact()
        self.sync()
        ids = self.ids()
        res = []
        for o in outs:
            a = np.empty(self.n)
            a[ids] = o.cpu().numpy()
            res.append(a)
        return tuple(res)


def _ids_of(scene, offset: int = 0) -> np.ndarray:
    ids = np.arange(offset, offset + scene.n, dtype=np.uint32)
    ids[scene.is_boundary] |= BOUNDARY_BIT
    return ids


class Simulation(_System):
    """One particle system.  Arrays come back in original particle order via
    :meth:`fetch`."""

    def __init__(self, scene, precision: str = "mixed", device: str = "cuda:0",
                 stream=None, c_mode: int = SPH_C_TAIT, delta_pairs: int = SPH_DELTA_FLUID,
                 scheme: int = SCHEME_VERLET):
        self.lib = load()
        self.params = make_params(scene.params, precision, c_mode=c_mode,
                                  delta_pairs=delta_pairs, scheme=scheme)
        check(self.lib.sph_check_params(C.byref(self.params)))
        nbytes = C.c_size_t(0)
        check(self.lib.sph_workspace_bytes(C.byref(self.params), scene.n, C.byref(nbytes)))
        self._alloc(scene.n, precision, device, stream, nbytes.value)
        check(self.lib.sph_workspace_init(C.byref(self.params), self.n, self.ws_ptr,
                                          self.ws_bytes, self._s()))
        self.upload(scene)

    def _set_density(self, ptr, which):
        check(self.lib.sph_set_density(C.byref(self.params), C.byref(self.state), ptr, which,
                                       self._s()))

    def _get_density(self, ptr, which):
        check(self.lib.sph_get_density(C.byref(self.params), C.byref(self.state), ptr, which,
                                       self._s()))

    def _interact(self, outs, mumax):
        check(self.lib.sph_interact(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                    *outs, mumax, self._s()))

    def upload(self, scene, prev=None) -> None:
        """Load a scene (original order).  `prev` optionally gives the
        previous Verlet level as a dict with ux, uy, uz, rho; by default it
        equals the current level."""
        pv = prev if prev is not None else dict(ux=scene.ux, uy=scene.uy, uz=scene.uz,
                                                rho=scene.rho)
        vals = dict(x=scene.x, y=scene.y, z=scene.z, ux=scene.ux, uy=scene.uy, uz=scene.uz,
                    uxm=pv["ux"], uym=pv["uy"], uzm=pv["uz"])
        self._upload_arrays(vals, _ids_of(scene), scene.rho, pv["rho"])

    # -- the four verbs ---------------------------------------------------
    def build_cells(self) -> None:
        check(self.lib.sph_build_cells(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                       self._s()))

    def neighbour_stats(self):
        """(fluid-neighbour count, boundary-neighbour count, id-set hash) per
        particle, numpy arrays in original particle order."""
        torch = self.torch
        if not self.state.cells_valid:
            self.build_cells()
        nf = torch.empty(self.n, dtype=torch.int32, device=self.dev)
        nb = torch.empty(self.n, dtype=torch.int32, device=self.dev)
        hs = torch.empty(self.n, dtype=torch.int32, device=self.dev)
        check(self.lib.sph_neighbour_stats(C.byref(self.params), C.byref(self.state),
                                           self.ws_ptr, nf.data_ptr(), nb.data_ptr(),
                                           hs.data_ptr(), self._s()))
        self.sync()
        ids = self.ids()
        out = []
        for t, dt in ((nf, np.int64), (nb, np.int64), (hs, np.uint32)):
            a = np.empty(self.n, dtype=dt)
            v = t.cpu().numpy()
            a[ids] = v.view(np.uint32) if dt is np.uint32 else v
            out.append(a)
        return tuple(out)

    def step(self, dt: float, step_index: int) -> None:
        check(self.lib.sph_step(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                float(dt), int(step_index), self._s()))

    def run(self, nsteps: int, dt: float, step0: int) -> None:
        check(self.lib.sph_run(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                               int(nsteps), float(dt), int(step0), self._s()))

    def run_noalloc(self, nsteps: int, dt: float, step0: int) -> None:
        """run() through sph_run_noalloc: the library's static scratch array
        instead of this system's workspace (whose clock it does not touch)."""
        check(self.lib.sph_run_noalloc(C.byref(self.params), C.byref(self.state), int(nsteps),
                                       float(dt), int(step0), self._s()))

    def run_profiled(self, nsteps: int, dt: float, step0: int, ev_begin, ev_end,
                     region: int = REGION_INTERACT) -> None:
        """run() recording hipEvent_t handles (ctypes arrays of c_void_p)
        around one region of every step."""
        check(self.lib.sph_run_profiled(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                        int(nsteps), float(dt), int(step0), int(region),
                                        ev_begin, ev_end, self._s()))

    def diagnostics(self, probes: Optional[Sequence[Sequence[float]]] = None):
        if not self.state.cells_valid:
            self.build_cells()
        pts = np.ascontiguousarray(np.asarray(probes if probes is not None else np.zeros((0, 3)),
                                              np.float64).reshape(-1))
        npts = pts.size // 3
        out = SphDiag()
        pp = np.zeros(max(npts, 1))
        check(self.lib.sph_diagnostics(
            C.byref(self.params), C.byref(self.state), self.ws_ptr,
            pts.ctypes.data if npts else None, npts, C.byref(out),
            pp.ctypes.data if npts else None, self._s()))
        return out.as_dict(), pp[:npts]


    def boundary_force(self, box):
        """(force vector, particle count) of the boundary particles inside
        box = (x0, x1, y0, y1, z0, z1)."""
        if not self.state.cells_valid:
            self.build_cells()
        b = np.ascontiguousarray(np.asarray(box, np.float64).reshape(6))
        f = np.zeros(3)
        cnt = C.c_int64(0)
        check(self.lib.sph_boundary_force(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                          b.ctypes.data, f.ctypes.data, C.byref(cnt), self._s()))
        return f, int(cnt.value)

    def probe_impulse(self, probes, reset: bool = False):
        """(probe pressures, pressure impulses since the last reset)."""
        if not self.state.cells_valid:
            self.build_cells()
        pts = np.ascontiguousarray(np.asarray(probes, np.float64).reshape(-1))
        npts = pts.size // 3
        pp = np.zeros(npts)
        ip = np.zeros(npts)
        check(self.lib.sph_probe_impulse(C.byref(self.params), C.byref(self.state), self.ws_ptr,
                                         pts.ctypes.data, npts, int(bool(reset)), pp.ctypes.data,
                                         ip.ctypes.data, self._s()))
        return pp, ip


    def mps_operators(self, re: float, l0: float, phi=None, beta1: float = 0.98,
                      rho1: float = 0.2, n0: Optional[float] = None,
                      lambda0: Optional[float] = None):
        """Explicit MPS operators (sph_mps_operators) at the current state:
        dict of pnd, lap, grad (3, n), sigma, surface, numpy in original
        particle order.  phi: numpy array in original order (or None)."""
        torch = self.torch
        if n0 is None or lambda0 is None:
            n0, lambda0 = mps_constants(l0, re)
        if not self.state.cells_valid:
            self.build_cells()
        self.sync()
        ids = self.ids()
        f64 = dict(dtype=torch.float64, device=self.dev)
        ph = None
        if phi is not None:
            ph = torch.from_numpy(np.ascontiguousarray(np.asarray(phi, np.float64)[ids])).to(
                self.dev)
        pnd = torch.empty(self.n, **f64)
        lap = torch.empty(self.n, **f64)
        grad = torch.empty(3 * self.n, **f64)
        sig = torch.empty(self.n, **f64)
        surf = torch.empty(self.n, dtype=torch.int32, device=self.dev)
        m = SphMps(float(re), float(n0), float(lambda0), float(beta1), float(rho1), float(l0))
        self.sync()
        check(self.lib.sph_mps_operators(
            C.byref(self.params), C.byref(self.state), self.ws_ptr, C.byref(m),
            ph.data_ptr() if ph is not None else None, pnd.data_ptr(),
            lap.data_ptr() if ph is not None else None,
            grad.data_ptr() if ph is not None else None, sig.data_ptr(), surf.data_ptr(),
            self._s()))
        self.sync()

        def orig(t):
            a = t.cpu().numpy()
            out = np.empty_like(a)
            out[ids] = a
            return out
        res = {"pnd": orig(pnd), "sigma": orig(sig), "surface": orig(surf)}
        if ph is not None:
            res["lap"] = orig(lap)
            g = grad.view(3, self.n)
            res["grad"] = np.stack([orig(g[k]) for k in range(3)])
        return res


class Ensemble(_System):
    """A batch of independent systems in one state (sph_batch_*).  Instance k
    owns original ids [offsets[k], offsets[k] + counts[k])."""

    def __init__(self, scenes, precision: str = "mixed", device: str = "cuda:0", stream=None,
                 c_mode: int = SPH_C_TAIT, delta_pairs: int = SPH_DELTA_FLUID,
                 scheme: int = SCHEME_VERLET):
        self.lib = load()
        k = len(scenes)
        self.ninst = k
        self._params = (SphParams * k)()
        for i, sc in enumerate(scenes):
            self._params[i] = make_params(sc.params, precision, c_mode=c_mode,
                                          delta_pairs=delta_pairs, scheme=scheme)
        self.counts = np.array([sc.n for sc in scenes], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)[:-1]]).astype(np.int64)
        self._counts = (C.c_int64 * k)(*[int(c) for c in self.counts])
        self.batch = SphBatch(k, 0, self._params, self._counts)
        nbytes = C.c_size_t(0)
        check(self.lib.sph_batch_workspace_bytes(C.byref(self.batch), C.byref(nbytes)))
        self._alloc(int(self.counts.sum()), precision, device, stream, nbytes.value)
        check(self.lib.sph_batch_workspace_init(C.byref(self.batch), self.ws_ptr,
                                                self.ws_bytes, self._s()))
        self.upload(scenes)

    def _set_density(self, ptr, which):
        check(self.lib.sph_batch_set_density(C.byref(self.batch), C.byref(self.state),
                                             self.ws_ptr, ptr, which, self._s()))

    def _get_density(self, ptr, which):
        check(self.lib.sph_batch_get_density(C.byref(self.batch), C.byref(self.state),
                                             self.ws_ptr, ptr, which, self._s()))

    def _interact(self, outs, mumax):
        check(self.lib.sph_batch_interact(C.byref(self.batch), C.byref(self.state),
                                          self.ws_ptr, *outs, mumax, self._s()))

    def upload(self, scenes) -> None:
        cat = lambda f: np.concatenate([np.asarray(getattr(sc, f), np.float64) for sc in scenes])
        vals = {k: cat(k) for k in ("x", "y", "z", "ux", "uy", "uz")}
        vals.update(uxm=vals["ux"], uym=vals["uy"], uzm=vals["uz"])
        ids = np.concatenate([_ids_of(sc, int(o)) for sc, o in zip(scenes, self.offsets)])
        rho = cat("rho")
        self._upload_arrays(vals, ids, rho, rho)

    def build_cells(self) -> None:
        check(self.lib.sph_batch_build_cells(C.byref(self.batch), C.byref(self.state),
                                             self.ws_ptr, self._s()))

    def run(self, nsteps: int, dt: float, step0: int, mode: int = 0) -> None:
        check(self.lib.sph_batch_run(C.byref(self.batch), C.byref(self.state), self.ws_ptr,
                                     int(nsteps), float(dt), int(step0), int(mode), self._s()))

    def run_profiled(self, nsteps: int, dt: float, step0: int, ev_begin, ev_end,
                     region: int = REGION_INTERACT, mode: int = 0) -> None:
        check(self.lib.sph_batch_run_profiled(C.byref(self.batch), C.byref(self.state),
                                              self.ws_ptr, int(nsteps), float(dt), int(step0),
                                              int(mode), int(region), ev_begin, ev_end,
                                              self._s()))

    def diagnostics(self):
        """One dict per instance."""
        if not self.state.cells_valid:
            self.build_cells()
        out = (SphDiag * self.ninst)()
        check(self.lib.sph_batch_diagnostics(C.byref(self.batch), C.byref(self.state),
                                             self.ws_ptr, out, self._s()))
        return [o.as_dict() for o in out]

    def split_by_instance(self, arr: np.ndarray):
        """Split an array in original-id order into per-instance pieces."""
        return [arr[o:o + c] for o, c in zip(self.offsets, self.counts)]
