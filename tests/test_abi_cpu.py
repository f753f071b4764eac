"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol the header declares, and rejects bad arguments before any launch."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2306_01959_amd import lib, scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcsph.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lib.LIB_PATH):
        from paper_2306_01959_amd import build
        build.build()
    return lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(sph_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_what_binding_exports():
    assert declared_functions() == sorted(lib.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in declared_functions():
        assert name in syms, name
        assert hasattr(L, name)


def test_version(L):
    assert L.sph_version() == 1


STRUCTS = (("sph_params", lib.SphParams), ("sph_state", lib.SphState),
           ("sph_diag", lib.SphDiag), ("sph_tuning", lib.SphTuning), ("sph_batch", lib.SphBatch))


def test_struct_layout_matches_header(tmp_path):
    """sizeof/offsetof of the ABI structs, compiled from the header with
    gcc, equal the binding's ctypes mirrors."""
    prog = tmp_path / "layout.c"
    checks = []
    for cname, py in STRUCTS:
        checks.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            checks.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "wcsph.h"\n'
                    "int main(void){" + "".join(checks) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)],
                   check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for cname, py in STRUCTS:
        assert int(got[cname]) == C.sizeof(py)
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def params(**over):
    p = lib.make_params(scene.make_params(0.02), "mixed")
    for k, v in over.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [
    ("h", 0.0), ("h", -1.0), ("dp", 0.0), ("rho0", 0.0), ("c0", -1.0), ("gamma", 0.5),
    ("alpha", -0.1), ("delta", 1.5), ("cfl", 0.0), ("cfl", 1.5), ("mass", 0.0),
    ("cell_size", 0.01), ("precision", 7), ("c_mode", 3), ("delta_pairs", 2),
    ("scheme", 2), ("h", float("nan")), ("eta2_coef", -1.0),
])
def test_bad_params_rejected(L, field, value):
    p = params(**{field: value})
    assert L.sph_check_params(C.byref(p)) == lib.SPH_E_INVAL
    assert L.sph_last_error().decode() != ""


def test_grid_too_large(L):
    p = params()
    p.dims[:] = [2048, 2048, 1024]
    assert L.sph_check_params(C.byref(p)) == lib.SPH_E_RANGE


def test_workspace_bytes(L):
    p = params()
    nb = C.c_size_t(0)
    assert L.sph_workspace_bytes(C.byref(p), 28392, C.byref(nb)) == 0
    assert nb.value > 28392 * 70 and nb.value % 256 == 0
    assert L.sph_workspace_bytes(C.byref(p), 0, C.byref(nb)) == lib.SPH_E_INVAL
    assert L.sph_workspace_bytes(C.byref(p), 1 << 31, C.byref(nb)) == lib.SPH_E_RANGE
    assert L.sph_workspace_bytes(None, 10, C.byref(nb)) == lib.SPH_E_INVAL
    p64 = lib.make_params(scene.make_params(0.02), "fp64")
    nb64 = C.c_size_t(0)
    L.sph_workspace_bytes(C.byref(p64), 28392, C.byref(nb64))
    assert nb64.value > nb.value


def test_calls_rejected_before_launch(L):
    """Null state, null workspace, misaligned workspace, stale cells: every
    entry point answers with an error code and launches nothing (no GPU is
    needed to see that)."""
    p = params()
    st = lib.SphState()
    assert L.sph_build_cells(C.byref(p), None, None, None) == lib.SPH_E_INVAL
    assert L.sph_build_cells(C.byref(p), C.byref(st), None, None) == lib.SPH_E_INVAL  # n = 0
    st.n = 100
    assert L.sph_build_cells(C.byref(p), C.byref(st), None, None) == lib.SPH_E_INVAL  # null arrays
    # fake but aligned non-null pointers: validation only, nothing is dereferenced
    fake = 1 << 20
    for k, _ in lib.SphState._fields_:
        if k not in ("n", "cells_valid", "reserved"):
            setattr(st, k, fake)
            fake += 1 << 20
    assert L.sph_build_cells(C.byref(p), C.byref(st), None, None) == lib.SPH_E_INVAL  # ws null
    assert L.sph_build_cells(C.byref(p), C.byref(st), 1 << 30 | 8, None) == lib.SPH_E_INVAL
    st.cells_valid = 0
    outs = [1 << 33] * 4
    assert L.sph_interact(C.byref(p), C.byref(st), 1 << 30, *outs, None, None) == lib.SPH_E_STATE
    assert L.sph_diagnostics(C.byref(p), C.byref(st), 1 << 30, None, 0, None, None,
                             None) == lib.SPH_E_INVAL
    d = lib.SphDiag()
    assert L.sph_diagnostics(C.byref(p), C.byref(st), 1 << 30, None, 0, C.byref(d), None,
                             None) == lib.SPH_E_STATE
    assert L.sph_diagnostics(C.byref(p), C.byref(st), 1 << 30, None, 5000, C.byref(d), None,
                             None) == lib.SPH_E_INVAL
    assert L.sph_step(C.byref(p), C.byref(st), 1 << 30, float("nan"), 0, None) == lib.SPH_E_INVAL
    assert L.sph_step(C.byref(p), C.byref(st), 1 << 30, 1e-4, -1, None) == lib.SPH_E_INVAL
    assert L.sph_run(C.byref(p), C.byref(st), 1 << 30, -1, 1e-4, 0, None) == lib.SPH_E_INVAL
    st.x = (1 << 20) + 4          # misaligned double array
    assert L.sph_build_cells(C.byref(p), C.byref(st), 1 << 30, None) == lib.SPH_E_INVAL
    assert "misaligned" in L.sph_last_error().decode()


def test_workspace_init_size_check(L):
    p = params()
    assert L.sph_workspace_init(C.byref(p), 100, 1 << 30, 64, None) == lib.SPH_E_SIZE


# ------------------------------------------------------------------ batch

def batch_of(plist, counts):
    arr = (lib.SphParams * len(plist))(*plist)
    cnt = (C.c_int64 * len(counts))(*counts)
    b = lib.SphBatch(len(plist), 0, arr, cnt)
    b._keep = (arr, cnt)
    return b


def test_batch_workspace_bytes(L):
    p1 = params()
    p2 = lib.make_params(scene.make_params(0.03, alpha=0.05), "mixed")
    b = batch_of([p1, p2], [5000, 3000])
    nb = C.c_size_t(0)
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == 0
    assert nb.value > 8000 * 70 and nb.value % 256 == 0
    # one more instance of the same grid adds at least its cell table
    b3 = batch_of([p1, p2, p1], [5000, 3000, 1])
    nb3 = C.c_size_t(0)
    assert L.sph_batch_workspace_bytes(C.byref(b3), C.byref(nb3)) == 0
    ncell = p1.dims[0] * p1.dims[1] * p1.dims[2]
    assert nb3.value >= nb.value + 4 * ncell


def test_batch_rejected_before_launch(L):
    p1 = params()
    p64 = lib.make_params(scene.make_params(0.02), "fp64")
    nb = C.c_size_t(0)
    assert L.sph_batch_workspace_bytes(None, C.byref(nb)) == lib.SPH_E_INVAL
    b = batch_of([p1, p64], [10, 10])
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_INVAL
    assert "precision" in L.sph_last_error().decode()
    b = batch_of([p1, p1], [10, 0])
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_INVAL
    b = batch_of([p1], [10])
    b.ninst = 0
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_INVAL
    b.ninst = lib.MAX_INSTANCES + 1
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_INVAL
    bad = params(h=-1.0)
    b = batch_of([p1, bad], [10, 10])
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_INVAL
    assert "instance 1" in L.sph_last_error().decode()
    b = batch_of([p1, p1], [1 << 30, 1 << 30])
    assert L.sph_batch_workspace_bytes(C.byref(b), C.byref(nb)) == lib.SPH_E_RANGE
    # state checks: n must equal the sum of the counts; run mode bits
    b = batch_of([p1, p1], [60, 40])
    st = lib.SphState()
    fake = 1 << 20
    for k, _ in lib.SphState._fields_:
        if k not in ("n", "cells_valid", "reserved"):
            setattr(st, k, fake)
            fake += 1 << 20
    st.n = 99
    assert L.sph_batch_build_cells(C.byref(b), C.byref(st), 1 << 30, None) == lib.SPH_E_INVAL
    st.n = 100
    assert L.sph_batch_run(C.byref(b), C.byref(st), 1 << 30, 1, 1e-4, 0, 4,
                           None) == lib.SPH_E_INVAL
    assert L.sph_batch_run(C.byref(b), C.byref(st), 1 << 30, 1, 1e-4, 0, lib.RUN_GRAPH,
                           None) == lib.SPH_E_INVAL
    assert "stream" in L.sph_last_error().decode()
    assert L.sph_batch_run_profiled(C.byref(b), C.byref(st), 1 << 30, 1, 1e-4, 0,
                                    lib.RUN_GRAPH, 0, None, None, 1 << 12) == lib.SPH_E_INVAL
    assert L.sph_batch_run_profiled(C.byref(b), C.byref(st), 1 << 30, 1, 1e-4, 0, 0, 9,
                                    None, None, None) == lib.SPH_E_INVAL
    st.cells_valid = 0
    d = (lib.SphDiag * 2)()
    assert L.sph_batch_diagnostics(C.byref(b), C.byref(st), 1 << 30, d,
                                   None) == lib.SPH_E_STATE
    outs = [1 << 33] * 4
    assert L.sph_batch_interact(C.byref(b), C.byref(st), 1 << 30, *outs, None,
                                None) == lib.SPH_E_STATE
    assert L.sph_batch_workspace_init(C.byref(b), 1 << 30, 64, None) == lib.SPH_E_SIZE


def test_loads_rejected_before_launch(L):
    """sph_boundary_force and sph_probe_impulse validate their arguments
    before touching the device (fake, aligned device pointers)."""
    import ctypes as C
    from paper_2306_01959_amd import lib, scene
    sc = scene.config_scene(1)
    p = lib.make_params(sc.params, "mixed")
    st = lib.SphState()
    st.n = sc.n
    for name, _ in lib.SphState._fields_[1:25]:
        setattr(st, name, 1 << 20)
    ws = C.c_void_p(1 << 24)
    f = (C.c_double * 3)()
    bad_box = (C.c_double * 6)(0.5, 0.4, 0.0, 1.0, 0.0, 1.0)       # lo > hi along x
    assert L.sph_boundary_force(C.byref(p), C.byref(st), ws, bad_box, f, None, None) == \
        lib.SPH_E_INVAL
    nan_box = (C.c_double * 6)(0.0, float("nan"), 0.0, 1.0, 0.0, 1.0)
    assert L.sph_boundary_force(C.byref(p), C.byref(st), ws, nan_box, f, None, None) == \
        lib.SPH_E_INVAL
    box = (C.c_double * 6)(0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    st.cells_valid = 0                                              # stale cells
    assert L.sph_boundary_force(C.byref(p), C.byref(st), ws, box, f, None, None) == \
        lib.SPH_E_STATE
    pts = (C.c_double * 3)(0.1, 0.1, 0.1)
    out = (C.c_double * 1)()
    imp = (C.c_double * 1)()
    assert L.sph_probe_impulse(C.byref(p), C.byref(st), ws, pts, 0, 0, out, imp, None) == \
        lib.SPH_E_INVAL
    assert L.sph_probe_impulse(C.byref(p), C.byref(st), ws, pts, 1, 2, out, imp, None) == \
        lib.SPH_E_INVAL
    assert L.sph_probe_impulse(C.byref(p), C.byref(st), ws, pts, 1, 0, out, imp, None) == \
        lib.SPH_E_STATE


def test_lagged_symplectic_batch_rejected(L):
    """The lagged fused step is the Verlet scheme's; a symplectic batch asking
    for it is rejected before anything is launched."""
    import ctypes as C
    from paper_2306_01959_amd import lib, scene
    scs = scene.ensemble(2, master_seed=21, dps=(0.05,))
    params = (lib.SphParams * 2)(*[lib.make_params(s.params, "mixed",
                                                   scheme=lib.SCHEME_SYMPLECTIC) for s in scs])
    counts = (C.c_int64 * 2)(*[s.n for s in scs])
    b = lib.SphBatch(2, 0, params, counts)
    st = lib.SphState()
    st.n = sum(s.n for s in scs)
    for name, _ in lib.SphState._fields_[1:25]:
        setattr(st, name, 1 << 20)
    ws = C.c_void_p(1 << 24)
    rc = L.sph_batch_run(C.byref(b), C.byref(st), ws, 5, -1.0, 0, lib.RUN_LAGGED, None)
    assert rc == lib.SPH_E_INVAL
    assert b"Verlet" in L.sph_last_error()
    # mixed schemes in one batch
    params[1] = lib.make_params(scs[1].params, "mixed")
    rc = L.sph_batch_run(C.byref(b), C.byref(st), ws, 5, -1.0, 0, 0, None)
    assert rc == lib.SPH_E_INVAL and b"scheme" in L.sph_last_error()


def test_mps_constants_match_oracle(L, oracle_lib):
    """sph_mps_constants runs on the host: n0 and lambda0 of the library equal
    the oracle's lattice sums (eq. mpslambda) for several radii."""
    from paper_2306_01959_amd import lib
    for l0, k in ((0.005, 2.1), (1.0, 3.1), (0.01, 4.0)):
        n0, lam = lib.mps_constants(l0, k * l0)
        on0, olam = oracle_lib.mps_lattice(l0, k * l0)
        assert n0 == pytest.approx(on0, rel=1e-14)
        assert lam == pytest.approx(olam, rel=1e-14)
    with pytest.raises(lib.SphError):
        lib.mps_constants(0.01, 0.0)
    with pytest.raises(lib.SphError):
        lib.mps_constants(0.01, 1.0)        # re > 64 l0


def test_mps_operators_rejected_before_launch(L):
    import ctypes as C
    from paper_2306_01959_amd import lib, scene
    sc = scene.config_scene(1)
    p = lib.make_params(sc.params, "fp64")
    st = lib.SphState()
    st.n = sc.n
    for name, _ in lib.SphState._fields_[1:25]:
        setattr(st, name, 1 << 20)
    st.cells_valid = 1
    ws = C.c_void_p(1 << 24)
    buf = C.c_void_p(1 << 22)
    good = lib.SphMps(0.9 * p.cell_size, 14.4, 1.7, 0.98, 0.2, 0.02)

    def call(m, phi=buf, lap=buf, grad=buf):
        return L.sph_mps_operators(C.byref(p), C.byref(st), ws, C.byref(m), phi, buf, lap,
                                   grad, buf, buf, None)
    bad = lib.SphMps(1.1 * p.cell_size, 14.4, 1.7, 0.98, 0.2, 0.02)     # re > cell
    assert call(bad) == lib.SPH_E_INVAL
    bad = lib.SphMps(0.9 * p.cell_size, 14.4, 1.7, 1.5, 0.2, 0.02)      # beta1 > 1
    assert call(bad) == lib.SPH_E_INVAL
    assert call(good, phi=None) == lib.SPH_E_INVAL                      # lap without phi
    st.cells_valid = 0
    assert call(good) == lib.SPH_E_STATE


def test_tuning_validated_and_reported(L):
    """sph_set_tuning is host-side: it accepts the documented values of every
    field, rejects anything else without changing the current setting, and
    sph_get_split reports the shape it set (no GPU needed)."""
    p = params()
    bad = [dict(split_mixed=2), dict(group_fp64=32), dict(kernel_mixed=9),
           dict(xcd_run_fp64=4), dict(xcd_run_mixed=-1), dict(xcd_run_mixed=64),
           dict(full_gather=2), dict(full_gather=-1)]
    try:
        lib.set_tuning(split_mixed=3, group_mixed=16, kernel_mixed=1, xcd_run_mixed=32)
        for kw in bad:
            with pytest.raises(lib.SphError) as e:
                lib.set_tuning(**kw)
            assert e.value.code == lib.SPH_E_INVAL, kw
        p.precision = lib.SPH_MIXED
        assert lib.get_split(p, 100000) == (3, 16, 1)
        for run in (0, 1, 8, 32):
            lib.set_tuning(xcd_run_fp64=run, xcd_run_mixed=run)
        for full in (0, 1):
            lib.set_tuning(full_gather=full)
    finally:
        lib.set_tuning()


def test_autotune_table_shapes():
    """Table entries of two, three and four values all name a full launch
    shape (kernel, waves per chunk, targets per group, XCD run), and every
    shipped entry is one the library accepts."""
    from paper_2306_01959_amd import autotune
    assert autotune.full_shape([3, 8]) == (1, 3, 8, 1)
    assert autotune.full_shape([2, 1, 16]) == (2, 1, 16, 1)
    assert autotune.full_shape([1, 1, 16, 32]) == (1, 1, 16, 32)
    tab = autotune._load()
    assert tab, "shipped table missing"
    try:
        for key, ent in tab.items():
            k, split, group, run = autotune.full_shape(ent["shape"])
            prec = key.split(":")[1] if key.startswith("ensemble") else key.split(":")[0]
            assert prec in ("mixed", "fp64"), key
            autotune.apply(prec, ent["shape"])      # raises SphError if rejected
            assert run in autotune.XCD_RUNS
    finally:
        autotune._state.update(fp64=(0, 0, 0, 0), mixed=(0, 0, 0, 0))
        lib.set_tuning()
