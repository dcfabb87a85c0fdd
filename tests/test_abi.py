"""CPU checks of the C ABI: libmpm.so loads, exports every function that
include/mpm.h declares, and rejects bad arguments on the host before any
device work (no compute call is made here)."""
import ctypes as C
import os
import re

import pytest

from paper_2102_01604_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mpm_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmpm.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "mpm_fit" in names and "mpm_uncertainty" in names and "mpm_simulate" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(_lib.SIGNATURES)


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes struct mirrors the header: size and each field offset, as
    gcc lays the C structs out."""
    import subprocess
    structs = {"mpm_protocol": _lib.mpm_protocol, "mpm_grid": _lib.mpm_grid, "mpm_options": _lib.mpm_options,
               "mpm_report": _lib.mpm_report, "mpm_kernel_stat": _lib.mpm_kernel_stat,
               "mpm_request": _lib.mpm_request, "mpm_space": _lib.mpm_space,
               "mpm_voxel_protocols": _lib.mpm_voxel_protocols, "mpm_rice_fit": _lib.mpm_rice_fit,
               "mpm_tune_result": _lib.mpm_tune_result}
    rename = {"lam": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpm.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            cf = rename.get(f[0], f[0])
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])


def _fit_raw(lib, proto, dims, opts):
    rep = _lib.mpm_report()
    return lib.mpm_fit(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid(dims)), 0,
                       C.c_void_p(16), None, C.byref(_lib.make_options(opts)), C.c_void_p(16),
                       C.byref(rep), None, 0, None)


@pytest.mark.parametrize("mutate,status", [
    (lambda p, d, o: p.update(tr=[0.0, 0.025, 0.025]), 1),
    (lambda p, d, o: p.update(flip=[0.1, 3.5, 0.1]), 1),
    (lambda p, d, o: p.update(sigma=[0.0] * 22), 1),
    (lambda p, d, o: p.update(te=[-1.0] + p["te"][1:]), 1),
    (lambda p, d, o: p.update(n_echoes=[0, 8, 6]), 1),
    (lambda p, d, o: p.update(mt=[0, 0, 0]), 2),
    (lambda p, d, o: d.__setitem__(0, 0), 1),
    (lambda p, d, o: o.update(n_gn=-1), 1),
    (lambda p, d, o: o.update(lam=[-1.0, 0, 0, 0]), 1),
    (lambda p, d, o: o.update(flags=3), 1),
    (lambda p, d, o: o.update(basis="rate"), 2),
    (lambda p, d, o: o.update(start_outer=1), 1),  # a MAP option
    (lambda p, d, o: o.update(mode="map", n_outer=3, start_outer=3), 1),
    (lambda p, d, o: o.update(mode="map", n_outer=3, start_outer=-1), 1),
    (lambda p, d, o: o.update(mode="map", n_outer=3, start_outer=1, tol_outer=0.1), 2),
    (lambda p, d, o: (d.__setitem__(0, 1), d.__setitem__(1, 1), d.__setitem__(2, 1), o.update(mode="map")), 2),
])
def test_host_validation(lib, mutate, status):
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    dims = [8, 8, 8]
    opts = {"mode": "ml", "n_gn": 5}
    mutate(proto, dims, opts)
    st = _fit_raw(lib, proto, dims, opts)
    assert st == status, lib.mpm_last_error()
    assert lib.mpm_last_error()


def test_unknown_loading_and_oversized_grid_rejected(lib):
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    o = _lib.make_options({"mode": "ml", "n_gn": 5})
    o.loading = 3
    rep = _lib.mpm_report()
    st = lib.mpm_fit(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid([8, 8, 8])), 0, C.c_void_p(16), None,
                     C.byref(o), C.c_void_p(16), C.byref(rep), None, 0, None)
    assert st == 1 and "loading" in lib.mpm_last_error().decode()
    # byte offsets into one image are 32-bit in the kernels: N < 2^30
    st = _fit_raw(lib, proto, [1024, 1024, 1024], {"mode": "ml", "n_gn": 5})
    assert st == 1 and "2^30" in lib.mpm_last_error().decode()


def test_projected_argument_validation(lib):
    """Spaces are checked on the host before any device work."""
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    eye = [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]]

    def run(spaces):
        rep = _lib.mpm_report()
        return lib.mpm_fit_projected(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid([8, 8, 8])),
                                     None if spaces is None else _lib.make_spaces(spaces), 0, C.c_void_p(16), None,
                                     C.byref(_lib.make_options({"mode": "map", "n_gn": 2})), C.c_void_p(16),
                                     C.byref(rep), None, 0, None)
    ok = {"dims": (8, 8, 8), "affine": eye}
    assert run(None) == 1
    for bad, what in (({"dims": (0, 8, 8), "affine": eye}, "axis"),
                      ({"dims": (8, 8, 8), "affine": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, float("nan"), 0]]}, "finite"),
                      ({"dims": (8, 8, 8), "affine": [[20, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]]}, "length"),
                      ({"dims": (8, 8, 8), "affine": [[1, 0, 0, 0], [1, 0, 0, 0], [0, 0, 1, 0]]}, "length"),
                      ({"dims": (8, 8, 8), "affine": [[1, 1, 0, 0], [1, 1, 0, 0], [0, 0, 1, 0]]}, "singular")):
        st = run([ok, bad, ok])
        assert st == 1 and what in lib.mpm_last_error().decode(), (what, lib.mpm_last_error())
    # the receive field is a reconstruction-grid option only
    o = _lib.make_options({"mode": "map", "n_gn": 2})
    o.b1_receive = 16
    rep = _lib.mpm_report()
    st = lib.mpm_fit_projected(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid([8, 8, 8])),
                               _lib.make_spaces([ok, ok, ok]), 0, C.c_void_p(16), None, C.byref(o), C.c_void_p(16),
                               C.byref(rep), None, 0, None)
    assert st == 2 and "b1_receive" in lib.mpm_last_error().decode()
    st = lib.mpm_uncertainty_projected(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid([8, 8, 8])),
                                       _lib.make_spaces([ok, ok, ok]), 0, C.c_void_p(16), None, C.byref(o),
                                       C.c_void_p(16), C.c_void_p(16), None, None)
    assert st == 2 and "b1_receive" in lib.mpm_last_error().decode()


def test_voxelwise_argument_validation(lib):
    """mpm_fit_voxelwise checks its arguments on the host before any device work."""
    fake = C.c_void_p(16)
    shape = {"n_echoes": [5, 5, 5], "mt": [0, 0, 1], "sigma": [1.0] * 15}

    def run(shape=shape, n=1000, opts=None, arrays=True, echoes=fake, receive=False):
        p = _lib.make_voxel_protocols(shape)
        if arrays:
            p.tr_s = p.flip_rad = p.te_s = 16
        o = _lib.make_options(opts if opts is not None else {"mode": "ml", "n_gn": 5, "init": "const",
                                                               "init_const": [0.0] * 4})
        if receive:
            o.b1_receive = 16
        rep = _lib.mpm_report()
        return lib.mpm_fit_voxelwise(C.byref(p), n, 0, echoes, C.byref(o), fake, None, None, C.byref(rep), None)

    cases = [
        (dict(arrays=False), 1, "device pointers"),
        (dict(echoes=None), 1, "device pointers"),
        (dict(n=0), 1, "n_voxels"),
        (dict(receive=True), 2, "b1_receive"),
        (dict(opts={"mode": "ml", "n_gn": 5, "init": "const", "init_const": [1.0, 1.0, 1.0, 1.5],
                    "basis": "rate"}), 1, "domain"),
        (dict(opts={"mode": "ml", "n_gn": 5, "init": "const", "init_const": [-1.0, 1.0, 1.0, 0.5],
                    "basis": "time"}), 1, "domain"),
        (dict(opts={"mode": "map", "n_gn": 5, "init": "const"}), 1, "ML fit"),
        (dict(opts={"mode": "ml", "n_gn": 5, "init": "default"}), 2, "one protocol"),
        (dict(opts={"mode": "ml", "n_gn": -1, "init": "const"}), 1, "n_gn"),
        (dict(opts={"mode": "ml", "n_gn": 5, "init": "const", "init_const": [float("nan"), 0, 0, 0]}), 1, "init_const"),
        (dict(shape={"n_echoes": [5, 5], "mt": [0, 0], "sigma": [1.0] * 10}), 2, "MT"),
        (dict(shape={"n_echoes": [5, 0, 5], "mt": [0, 0, 1], "sigma": [1.0] * 10}), 1, "echoes"),
        (dict(shape={"n_echoes": [5, 5, 5], "mt": [0, 0, 1], "sigma": [1.0] * 14 + [0.0]}), 1, "sigma"),
        (dict(shape={"n_echoes": [5] * 9, "mt": [0] * 8 + [1], "sigma": [1.0] * 45}), 1, "n_contrasts"),
    ]
    for kw, status, what in cases:
        st = run(**kw)
        assert st == status and what in lib.mpm_last_error().decode(), (kw, st, lib.mpm_last_error())


def test_unknown_basis_rejected(lib):
    o = _lib.make_options({"mode": "ml", "n_gn": 5, "init": "const", "init_const": [1.0, 1.0, 1.0, 0.5]})
    o.basis = 3
    p = _lib.make_voxel_protocols({"n_echoes": [5, 5, 5], "mt": [0, 0, 1], "sigma": [1.0] * 15})
    p.tr_s = p.flip_rad = p.te_s = 16
    rep = _lib.mpm_report()
    st = lib.mpm_fit_voxelwise(C.byref(p), 1000, 0, C.c_void_p(16), C.byref(o), C.c_void_p(16), None, None,
                               C.byref(rep), None)
    assert st == 1 and "basis" in lib.mpm_last_error().decode()
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    st = lib.mpm_fit(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid([8, 8, 8])), 0, C.c_void_p(16),
                     None, C.byref(o), C.c_void_p(16), C.byref(rep), None, 0, None)
    assert st == 1 and "basis" in lib.mpm_last_error().decode()


def test_noise_estimation_argument_validation(lib):
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    out = [(C.c_double * 22)(), (C.c_double * 3)(), (C.c_double * 22)(), (C.c_double * 4)()]

    def run(nbins=1024, n_iter=200, echoes=C.c_void_p(16), outs=out, p=proto):
        return lib.mpm_estimate_noise(C.byref(_lib.make_protocol(p)), C.byref(_lib.make_grid([8, 8, 8])), 0,
                                      echoes, None, nbins, n_iter, *outs, None, None, None)
    for kw, status, what in ((dict(nbins=8), 1, "nbins"), (dict(nbins=5000), 1, "nbins"), (dict(n_iter=-1), 1, "n_iter"),
                             (dict(echoes=None), 1, "echoes"), (dict(outs=[None] + out[1:]), 1, "host"),
                             (dict(p=dict(proto, mt=[0, 0, 0])), 2, "MT")):
        st = run(**kw)
        assert st == status and what in lib.mpm_last_error().decode(), (kw, st, lib.mpm_last_error())


def test_autotune_argument_validation(lib):
    for dims, reps, what in (((0, 8, 8), 5, "axis"), ((1, 1, 1), 5, "2 voxels"), ((8, 8, 8), 0, "reps")):
        st = lib.mpm_autotune(C.byref(_lib.make_grid(dims)), reps, None, None)
        assert st == 1 and what in lib.mpm_last_error().decode(), (dims, reps, lib.mpm_last_error())


def test_autotune_set_validation(lib):
    g = C.byref(_lib.make_grid((8, 8, 8)))
    for cg, col, what in ((-1, 0, "cg_workgroups"), (1 << 21, 0, "cg_workgroups"), (0, -5, "column_workgroups")):
        st = lib.mpm_autotune_set(g, cg, col)
        assert st == 1 and what in lib.mpm_last_error().decode(), (cg, col, lib.mpm_last_error())
    assert lib.mpm_autotune_set(C.byref(_lib.make_grid((0, 8, 8))), 16, 16) == 1
    assert lib.mpm_autotune_set(g, 16, 64) == 0  # host bookkeeping only
    lib.mpm_autotune_clear()


def test_null_pointers_rejected(lib):
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    rep = _lib.mpm_report()
    st = lib.mpm_fit(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid((4, 4, 4))), 0, None, None,
                     C.byref(_lib.make_options({})), None, C.byref(rep), None, 0, None)
    assert st == 1
    st = lib.mpm_simulate(C.byref(_lib.make_protocol(proto)), C.byref(_lib.make_grid((4, 4, 4))), None, None,
                          None, 0, None, None)
    assert st == 1


def test_footprint_is_host_only(lib):
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    ml = _lib.mpm_footprint_bytes(proto, (192, 240, 256), 0, 0)
    mp = _lib.mpm_footprint_bytes(proto, (192, 240, 256), 0, 1)
    N = 192 * 240 * 256
    assert ml >= N * (22 * 4 + 16)
    assert mp > ml
    assert _lib.mpm_footprint_bytes(proto, (192, 240, 256), 1, 1) < mp
    assert _lib.mpm_version().startswith("libmpm")
