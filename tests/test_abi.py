"""The C-ABI library on the CPU: it loads, exports every function include/picmcc.h
declares, its structs have the C compiler's layout in the Python binding, and
the host-only paths (footprints, validation) behave as documented.  No compute
call is made here."""
import ctypes as C
import os
import re
import subprocess

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "picmcc.h")


@pytest.fixture(scope="module")
def pm():
    import paper_1607_04069_amd as mod
    return mod


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(pm_\w+)\s*\(", txt, re.M)))


def test_every_declared_function_is_exported(pm):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", pm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pm_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    lib = C.CDLL(pm.LIB_PATH)
    for n in names:
        assert getattr(lib, n) is not None


def STRUCTS(mod):
    return (mod.pm_xsec, mod.pm_case_params, mod.pm_diagnostics, mod.pm_phase_sample, mod.pm_particles, mod.pm_fields,
            mod.pm_launch_shape, mod.pm_sputter_params, mod.pm_tp_source, mod.pm_tp_params, mod.pm_tp_trace,
            mod.pm_tp_result)


def _c_layout(tmp_path):
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "picmcc.h"', "int main(void){"]
    import paper_1607_04069_amd as mod
    for cls in STRUCTS(mod):
        t = cls.__name__
        lines.append(f'printf("{t} %zu\\n", sizeof({t}));')
        for f in cls._fields_:
            lines.append(f'printf("{t}.{f[0]} %zu\\n", offsetof({t}, {f[0]}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return dict(line.rsplit(" ", 1) for line in out.strip().splitlines())


def test_struct_layouts_match_c(pm, tmp_path):
    c = _c_layout(tmp_path)
    for cls in STRUCTS(pm):
        t = cls.__name__
        assert int(c[t]) == C.sizeof(cls), t
        for f in cls._fields_:
            assert int(c[f"{t}.{f[0]}"]) == getattr(cls, f[0]).offset, (t, f[0])


def test_footprint_and_validation(pm):
    p = pm.case_params(W.discharge_working())
    big = pm.pm_case_footprint(C.byref(p))
    # 8 particle arrays of 4 B, 2 of 8 B and 2 of 4 B per slot, two buffers, 4M slots per species
    assert big > 2 * 2 * 4_000_000 * 28
    for bad in (dict(n_cells=0), dict(n_cells=1025), dict(steps_per_cycle=0), dict(np_e=0),
                dict(capacity_e=10), dict(fp64=3), dict(gap_m=-1.0), dict(sort_interval=-2),
                dict(n_phase=-1), dict(n_phase=129), dict(n_phase=8, steps_per_cycle=4),
                dict(flux_profiles=2)):
        q = pm.case_params(dict(W.discharge_small(), **bad))
        assert pm.pm_case_footprint(C.byref(q)) == 0, bad
    small = pm.case_params(W.discharge_small())
    n = pm.pm_case_footprint(C.byref(small))
    # phase bins and flux sums: 16 B per node and species per bin, plus per-bin scalars
    nodes = W.discharge_small()["n_cells"] + 1
    more = pm.case_params(dict(W.discharge_small(), n_phase=10, flux_profiles=1))
    assert pm.pm_case_footprint(C.byref(more)) >= n + 2 * 10 * 2 * nodes * 16
    h = C.c_void_p()
    # rejected before any device access: a null arena, a short arena, a misaligned arena
    assert pm.pm_init_case(C.byref(small), None, n, None, C.byref(h)) == -1
    assert pm.pm_init_case(C.byref(small), C.c_void_p(1 << 20), n - 1, None, C.byref(h)) == -2
    assert pm.pm_init_case(C.byref(small), C.c_void_p((1 << 20) + 8), n, None, C.byref(h)) == -1
    assert h.value is None
    for code in range(-6, 1):
        assert pm.pm_status_string(code)
    # checkpoint calls without a case are rejected before any device access
    buf = (C.c_uint8 * 64)()
    assert pm.pm_checkpoint_bytes(None) == 0
    assert pm.pm_save_checkpoint(None, C.cast(buf, C.c_void_p), 64, None) == -1
    assert pm.pm_load_checkpoint(None, C.cast(buf, C.c_void_p), 64, None) == -1
    # the generator check: argument errors, and an empty request, never touch a device
    assert pm.pm_philox_words(0, 0, 0, 0, 0, 0, -1, None, None) == -1
    assert pm.pm_philox_words(0, 0, 0, 0, 0, 0, 5, None, None) == -1
    assert pm.pm_philox_words(0, 0, 0, 0, 0, 0, 0, None, None) == 0


def test_tp_validation(pm):
    src, tp = W.sputter_transport()
    tpp = pm.tp_params(tp)
    assert pm.pm_tp_footprint(C.byref(tpp)) > 0
    res = pm.pm_tp_result()
    cs = pm.tp_source(src)
    for bad in (dict(omega=0.3), dict(mode=7), dict(e_max=0), dict(gap_m=0.0)):
        q = pm.tp_params(dict(tp, **bad))
        assert pm.pm_run_test_particles(C.byref(q), C.byref(cs), C.c_void_p(1 << 20), 1 << 20, None,
                                        C.byref(res)) == -1
    assert pm.pm_run_test_particles(C.byref(tpp), C.byref(cs), C.c_void_p(1 << 20), 16, None,
                                    C.byref(res)) == -2
    # the form without an arena: invalid arguments and tallies beyond its static
    # scratch are rejected before any device access
    for bad in (dict(omega=0.3), dict(n_xbins=5000)):
        q = pm.tp_params(dict(tp, **bad))
        assert pm.pm_run_test_particles_static(C.byref(q), C.byref(cs), None, C.byref(res)) == -1
    big = pm.tp_params(dict(tp, n_ebins=200_000))
    assert pm.pm_tp_footprint(C.byref(big)) > pm.TP_STATIC_BYTES
    assert pm.pm_run_test_particles_static(C.byref(big), C.byref(cs), None, C.byref(res)) == -2


def test_batch_and_shape_validation(pm):
    """Rejected before any device access: no cases, a null handle, a bad shape."""
    none = (C.c_void_p * 1)(None)
    assert pm.pm_batch_footprint(None, 0) == 0
    assert pm.pm_batch_footprint(none, 1) == 0
    assert pm.pm_batch_footprint(none, 0) == 0
    h = C.c_void_p()
    assert pm.pm_batch_create(none, 1, C.c_void_p(1 << 20), 1 << 20, None, C.byref(h)) == -1
    assert h.value is None
    sh = pm.pm_launch_shape(unroll=8, waves=0, work_groups=0, deposit_mode=1, sort_interval=25, lanes=1)
    assert pm.pm_set_launch_shape(None, C.byref(sh), None) == -1
    assert pm.pm_batch_set_launch_shape(None, C.byref(sh), None) == -1
    assert pm.pm_get_launch_shape(None, C.byref(sh)) == -1
    assert pm.pm_batch_step(None, 1, None) == -1
    assert pm.pm_batch_step_rf_cycles(None, 1, None) == -1
