"""Python binding of libpicmcc (include/picmcc.h): argument marshalling only.

Every step of the PIC/MCC cycle and of the test-particle flight runs in the HIP
kernels of the library; this module converts parameter dicts to the C structs,
lets torch allocate the device arena and supply the stream, and copies results
into numpy arrays.  The C entry points are exposed under their own names
(``pm_init_case``, ``pm_step_rf_cycles``, ``pm_sample_diagnostics``,
``pm_inject_sputtered``, ``pm_run_test_particles`` ...) and wrapped by the small
``Case`` class and ``run_test_particles`` function.

Loading fails loudly when the library has not been built: there is no CPU path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpicmcc.so")

# ------------------------------------------------------------------ C structs
c_double_p = C.POINTER(C.c_double)
c_u64_p = C.POINTER(C.c_uint64)
c_i64_p = C.POINTER(C.c_int64)
c_u32_p = C.POINTER(C.c_uint32)
c_i32_p = C.POINTER(C.c_int32)
c_float_p = C.POINTER(C.c_float)


class pm_xsec(C.Structure):
    _fields_ = [("sigma_el", C.c_double), ("eth_exc", C.c_double), ("sigma0_exc", C.c_double),
                ("eth_ion", C.c_double), ("sigma0_ion", C.c_double), ("sigma_cx", C.c_double)]


class pm_case_params(C.Structure):
    _fields_ = [("gap_m", C.c_double), ("n_cells", C.c_int32), ("steps_per_cycle", C.c_int32),
                ("freq_hz", C.c_double), ("v0_volt", C.c_double), ("phase_rad", C.c_double),
                ("p_pa", C.c_double), ("t_gas_k", C.c_double), ("n0_m3", C.c_double),
                ("np_e", C.c_int64), ("np_i", C.c_int64), ("te_ev", C.c_double), ("ti_ev", C.c_double),
                ("capacity_e", C.c_int64), ("capacity_i", C.c_int64),
                ("ecap_e_ev", C.c_double), ("ecap_i_ev", C.c_double), ("xs", pm_xsec),
                ("seed", C.c_uint64), ("case_id", C.c_uint32), ("flags", C.c_uint32),
                ("fp64", C.c_int32), ("sort_interval", C.c_int32),
                ("v2_volt", C.c_double), ("phase2_rad", C.c_double), ("cb_f_m2", C.c_double),
                ("n_phase", C.c_int32), ("flux_profiles", C.c_int32)]


class pm_diagnostics(C.Structure):
    _fields_ = [("ne", c_double_p), ("ni", c_double_p), ("phi", c_double_p),
                ("iedf", c_u64_p), ("iadf", c_u64_p),
                ("step", C.c_int64), ("status", C.c_int32), ("warnings", C.c_uint32),
                ("n_e", C.c_int64), ("n_i", C.c_int64), ("avg_steps", C.c_int64),
                ("absorbed", (C.c_uint64 * 2) * 2), ("flux", (C.c_double * 2) * 2),
                ("mean_ion_energy", C.c_double * 2), ("collisions", C.c_uint64 * 5),
                ("candidates", C.c_uint64 * 2), ("overflow", C.c_uint64 * 2),
                ("births", C.c_uint64), ("particle_steps", C.c_uint64),
                ("gamma_e", c_double_p), ("gamma_i", c_double_p), ("u_e", c_double_p), ("u_i", c_double_p),
                ("iead", c_u64_p)]


class pm_phase_sample(C.Structure):
    _fields_ = [("ne", c_double_p), ("ni", c_double_p), ("phi", c_double_p),
                ("gamma_e", c_double_p), ("gamma_i", c_double_p), ("u_e", c_double_p), ("u_i", c_double_p),
                ("n_steps", C.c_int64), ("n_flux_samples", C.c_int64), ("status", C.c_int32)]


class pm_launch_shape(C.Structure):
    _fields_ = [("unroll", C.c_int32), ("waves", C.c_int32), ("work_groups", C.c_int32),
                ("deposit_mode", C.c_int32), ("sort_interval", C.c_int32), ("lanes", C.c_int32)]


SHAPE_KEYS = ("unroll", "waves", "work_groups", "deposit_mode", "sort_interval", "lanes")


class pm_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64), ("xt", c_double_p), ("ux", c_double_p),
                ("uy", c_double_p), ("uz", c_double_p), ("id", c_u64_p), ("next", c_u32_p)]


class pm_fields(C.Structure):
    _fields_ = [("qe", c_i64_p), ("qi", c_i64_p), ("phi", c_double_p), ("efield", c_double_p),
                ("sigma_init", C.c_double), ("n_absorbed_net", C.c_int64)]


class pm_sputter_params(C.Structure):
    _fields_ = [("yield_const", C.c_double), ("n_table", C.c_int32), ("table_e_ev", c_double_p),
                ("table_y", c_double_p), ("u_s_ev", C.c_double), ("e_cut_ev", C.c_double),
                ("n_atoms", C.c_int64), ("seed", C.c_uint64), ("job_id", C.c_uint32),
                ("electrode", C.c_int32), ("since_last", C.c_int32)]


class pm_tp_source(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("first_atom", C.c_int64), ("n_impacts", C.c_int64),
                ("n_emitted", C.c_int64), ("flux_m2s", C.c_double), ("u_s_ev", C.c_double),
                ("e_cut_ev", C.c_double), ("seed", C.c_uint64), ("job_id", C.c_uint32),
                ("electrode", C.c_int32)]


class pm_tp_params(C.Structure):
    _fields_ = [("p_pa", C.c_double), ("t_gas_k", C.c_double), ("d_ref", C.c_double),
                ("omega", C.c_double), ("t_ref", C.c_double), ("m_test_amu", C.c_double),
                ("m_gas_amu", C.c_double), ("gap_m", C.c_double), ("lateral_m", C.c_double),
                ("mode", C.c_int32), ("e_max", C.c_int64), ("n_ebins", C.c_int32),
                ("ebin_ev", C.c_double), ("n_tbins", C.c_int32), ("tbin_s", C.c_double),
                ("n_xbins", C.c_int32), ("scatter", C.c_int32), ("dt_s", C.c_double)]


class pm_tp_trace(C.Structure):
    _fields_ = [("wall", c_i32_p), ("events", c_u32_p), ("energy_ev", c_float_p),
                ("theta_deg", c_float_p), ("tof_s", c_float_p), ("vx", c_float_p),
                ("vy", c_float_p), ("vz", c_float_p)]


class pm_tp_result(C.Structure):
    _fields_ = [("e_hist", c_u64_p), ("theta_hist", c_u64_p), ("tof_hist", c_u64_p),
                ("trace", C.POINTER(pm_tp_trace)), ("time_s", c_double_p), ("disp_m", c_double_p),
                ("n_substrate", C.c_int64), ("n_target", C.c_int64), ("n_unfinished", C.c_int64),
                ("events", C.c_uint64), ("collisions", C.c_uint64), ("overflow", C.c_uint64),
                ("e_sum_substrate", C.c_double), ("e_sum_target", C.c_double), ("eta", C.c_double),
                ("deposition_flux", C.c_double), ("nu_max", C.c_double),
                ("density_m3", c_double_p), ("mean_vx", c_double_p)]


TP_STATIC_BYTES = 1 << 20      # PM_TP_STATIC_BYTES
STATUS = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_ENOSPACE", -3: "PM_EDEVICE", -4: "PM_ECAPACITY",
          -5: "PM_ENUMERIC", -6: "PM_ESTATE"}
N_ANGLE_BINS = 360
TP_THETA_BINS = 90
IEAD_E_GROUP = 4
IEAD_A_BINS = 90


class PicMccError(RuntimeError):
    def __init__(self, status, call):
        self.status = status
        super().__init__(f"{call} returned {STATUS.get(status, status)}: "
                         f"{_lib.pm_status_string(status).decode()}")


# ------------------------------------------------------------------ loading
def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1607_04069_amd/build.py` (there is no CPU fallback)")
    # torch ships its own HIP runtime; load it first so that the library binds to
    # the same one (device pointers and streams are per runtime instance: a
    # second runtime loaded from /opt/rocm would reject torch's)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "pm_status_string": (C.c_char_p, [C.c_int]),
        "pm_case_footprint": (C.c_size_t, [C.POINTER(pm_case_params)]),
        "pm_init_case": (C.c_int, [C.POINTER(pm_case_params), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "pm_step_rf_cycles": (C.c_int, [vp, C.c_int32, vp]),
        "pm_step": (C.c_int, [vp, C.c_int64, vp]),
        "pm_sample_diagnostics": (C.c_int, [vp, C.POINTER(pm_diagnostics), C.c_int32, vp]),
        "pm_sample_phase": (C.c_int, [vp, C.c_int32, C.POINTER(pm_phase_sample), vp]),
        "pm_diag_sizes": (C.c_int, [vp, c_i32_p, c_i32_p]),
        "pm_get_particles": (C.c_int, [vp, C.c_int32, C.POINTER(pm_particles), vp]),
        "pm_set_particles": (C.c_int, [vp, C.c_int32, C.POINTER(pm_particles), vp]),
        "pm_philox_words": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                      C.c_int64, vp, vp]),
        "pm_checkpoint_bytes": (C.c_size_t, [vp]),
        "pm_save_checkpoint": (C.c_int, [vp, vp, C.c_size_t, vp]),
        "pm_load_checkpoint": (C.c_int, [vp, vp, C.c_size_t, vp]),
        "pm_get_fields": (C.c_int, [vp, C.POINTER(pm_fields), vp]),
        "pm_case_info": (C.c_int, [vp, c_double_p, c_double_p, c_double_p, c_double_p, c_double_p]),
        "pm_destroy_case": (None, [vp]),
        "pm_get_step_profile": (C.c_int, [vp, c_u64_p, C.c_int64, c_i32_p, vp]),
        "pm_inject_sputtered": (C.c_int, [vp, C.POINTER(pm_sputter_params), C.POINTER(pm_tp_source), vp]),
        "pm_tp_footprint": (C.c_size_t, [C.POINTER(pm_tp_params)]),
        "pm_run_test_particles": (C.c_int, [C.POINTER(pm_tp_params), C.POINTER(pm_tp_source), vp,
                                            C.c_size_t, vp, C.POINTER(pm_tp_result)]),
        "pm_run_test_particles_static": (C.c_int, [C.POINTER(pm_tp_params), C.POINTER(pm_tp_source), vp,
                                                   C.POINTER(pm_tp_result)]),
        "pm_get_launch_shape": (C.c_int, [vp, C.POINTER(pm_launch_shape)]),
        "pm_set_launch_shape": (C.c_int, [vp, C.POINTER(pm_launch_shape), vp]),
        "pm_batch_get_launch_shape": (C.c_int, [vp, C.POINTER(pm_launch_shape)]),
        "pm_batch_set_launch_shape": (C.c_int, [vp, C.POINTER(pm_launch_shape), vp]),
        "pm_batch_footprint": (C.c_size_t, [C.POINTER(vp), C.c_int32]),
        "pm_batch_create": (C.c_int, [C.POINTER(vp), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "pm_batch_slots_footprint": (C.c_size_t, [C.c_int32, C.c_int32]),
        "pm_batch_create_slots": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, C.c_size_t, vp,
                                            C.POINTER(vp)]),
        "pm_batch_set_slot": (C.c_int, [vp, C.c_int32, vp, vp]),
        "pm_batch_step": (C.c_int, [vp, C.c_int64, vp]),
        "pm_batch_step_rf_cycles": (C.c_int, [vp, C.c_int32, vp]),
        "pm_batch_info": (C.c_int, [vp, c_i32_p, c_i32_p, c_i32_p]),
        "pm_batch_destroy": (None, [vp]),
        "pm_time_kernels": (C.c_int, [vp, C.c_int32, vp, c_double_p, c_double_p]),
        "pm_batch_time_kernels": (C.c_int, [vp, C.c_int32, vp, c_double_p, c_double_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
for _n in ("pm_status_string", "pm_case_footprint", "pm_init_case", "pm_step_rf_cycles", "pm_step",
           "pm_sample_diagnostics", "pm_sample_phase", "pm_diag_sizes", "pm_get_particles", "pm_set_particles",
           "pm_get_fields", "pm_case_info", "pm_destroy_case", "pm_inject_sputtered",
           "pm_checkpoint_bytes", "pm_save_checkpoint", "pm_load_checkpoint", "pm_philox_words",
           "pm_tp_footprint", "pm_run_test_particles", "pm_run_test_particles_static", "pm_get_step_profile", "pm_batch_footprint",
           "pm_batch_create", "pm_batch_step", "pm_batch_step_rf_cycles", "pm_batch_info",
           "pm_batch_slots_footprint", "pm_batch_create_slots", "pm_batch_set_slot",
           "pm_batch_destroy", "pm_get_launch_shape", "pm_set_launch_shape", "pm_batch_get_launch_shape",
           "pm_batch_set_launch_shape", "pm_time_kernels", "pm_batch_time_kernels"):
    globals()[_n] = getattr(_lib, _n)


def _check(status, call):
    if status != 0:
        raise PicMccError(status, call)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def case_params(p):
    """pm_case_params from a parameter dict (the workload/oracle field names)."""
    xs = pm_xsec(**{k: float(p[k]) for k in ("sigma_el", "eth_exc", "sigma0_exc", "eth_ion",
                                              "sigma0_ion", "sigma_cx")})
    return pm_case_params(
        gap_m=p["gap_m"], n_cells=p["n_cells"], steps_per_cycle=p["steps_per_cycle"],
        freq_hz=p["freq_hz"], v0_volt=p["v0_volt"], phase_rad=p["phase_rad"], p_pa=p["p_pa"],
        t_gas_k=p["t_gas_k"], n0_m3=p["n0_m3"], np_e=p["np_e"], np_i=p["np_i"], te_ev=p["te_ev"],
        ti_ev=p["ti_ev"], capacity_e=p["capacity_e"], capacity_i=p["capacity_i"],
        ecap_e_ev=p["ecap_e_ev"], ecap_i_ev=p["ecap_i_ev"], xs=xs, seed=p["seed"],
        case_id=p["case_id"], flags=p.get("flags", 0), fp64=int(p.get("fp64", 0)),
        sort_interval=int(p.get("sort_interval", 25)), v2_volt=float(p.get("v2_volt", 0.0)),
        phase2_rad=float(p.get("phase2_rad", 0.0)), cb_f_m2=float(p.get("cb_f_m2", 0.0)),
        n_phase=int(p.get("n_phase", 0)), flux_profiles=int(p.get("flux_profiles", 0)))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _arena(nbytes):
    import torch
    # 256-byte aligned device bytes owned by the caller (torch's allocator aligns to 512)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Case:
    """One discharge case resident in a torch-allocated device arena."""

    def __init__(self, p, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("picmcc needs a GPU (no CPU path)")
        self.p = dict(p)
        self._cp = case_params(self.p)
        nbytes = pm_case_footprint(C.byref(self._cp))
        if nbytes == 0:
            raise PicMccError(-1, "pm_case_footprint")
        self.arena = _arena(nbytes)
        self.stream = stream
        h = C.c_void_p()
        _check(pm_init_case(C.byref(self._cp), C.c_void_p(self.arena.data_ptr()), nbytes,
                            _stream(stream), C.byref(h)), "pm_init_case")
        self.h = h
        nodes, nb = C.c_int32(), C.c_int32()
        pm_diag_sizes(self.h, C.byref(nodes), C.byref(nb))
        self.nodes, self.n_ebins = nodes.value, nb.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            pm_destroy_case(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step_rf_cycles(self, n):
        _check(pm_step_rf_cycles(self.h, int(n), _stream(self.stream)), "pm_step_rf_cycles")

    def time_kernels(self, n):
        """Average (push, collision) launch durations in ms over n single steps."""
        a, b = C.c_double(), C.c_double()
        _check(pm_time_kernels(self.h, int(n), _stream(self.stream), C.byref(a), C.byref(b)), "pm_time_kernels")
        return a.value, b.value

    def launch_shape(self):
        sh = pm_launch_shape()
        _check(pm_get_launch_shape(self.h, C.byref(sh)), "pm_get_launch_shape")
        return {k: getattr(sh, k) for k in SHAPE_KEYS}

    def set_launch_shape(self, **kw):
        """Change any of unroll, waves, work_groups, deposit_mode, sort_interval."""
        cur = self.launch_shape()
        cur.update(kw)
        sh = pm_launch_shape(**{k: int(cur[k]) for k in SHAPE_KEYS})
        _check(pm_set_launch_shape(self.h, C.byref(sh), _stream(self.stream)), "pm_set_launch_shape")

    def step(self, n):
        _check(pm_step(self.h, int(n), _stream(self.stream)), "pm_step")

    def info(self):
        dx, dt, w = C.c_double(), C.c_double(), C.c_double()
        nu = (C.c_double * 2)()
        pt = (C.c_double * 2)()
        _check(pm_case_info(self.h, C.byref(dx), C.byref(dt), C.byref(w), nu, pt), "pm_case_info")
        return dict(dx=dx.value, dt=dt.value, w=w.value, nu_max=tuple(nu), p_tot=tuple(pt))

    def sample_diagnostics(self, reset=False):
        n, nb = self.nodes, self.n_ebins
        ne, ni, phi = np.zeros(n), np.zeros(n), np.zeros(n)
        iedf = np.zeros((2, nb), dtype=np.uint64)
        iadf = np.zeros((2, N_ANGLE_BINS), dtype=np.uint64)
        ge, gi, ue, ui = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
        iead = np.zeros((2, -(-nb // IEAD_E_GROUP), IEAD_A_BINS), dtype=np.uint64)
        d = pm_diagnostics(ne=_ptr(ne, C.c_double), ni=_ptr(ni, C.c_double), phi=_ptr(phi, C.c_double),
                           iedf=_ptr(iedf, C.c_uint64), iadf=_ptr(iadf, C.c_uint64),
                           gamma_e=_ptr(ge, C.c_double), gamma_i=_ptr(gi, C.c_double),
                           u_e=_ptr(ue, C.c_double), u_i=_ptr(ui, C.c_double), iead=_ptr(iead, C.c_uint64))
        _check(pm_sample_diagnostics(self.h, C.byref(d), int(bool(reset)), _stream(self.stream)),
               "pm_sample_diagnostics")
        return dict(step=d.step, status=d.status, warnings=d.warnings, n_e=d.n_e, n_i=d.n_i,
                    avg_steps=d.avg_steps, ne=ne, ni=ni, phi=phi, iedf=iedf, iadf=iadf,
                    absorbed=np.array([[d.absorbed[s][e] for e in range(2)] for s in range(2)]),
                    flux=np.array([[d.flux[s][e] for e in range(2)] for s in range(2)]),
                    mean_ion_energy=np.array(list(d.mean_ion_energy)),
                    collisions=np.array(list(d.collisions)), candidates=np.array(list(d.candidates)),
                    overflow=np.array(list(d.overflow)), births=d.births,
                    particle_steps=d.particle_steps, gamma_e=ge, gamma_i=gi, u_e=ue, u_i=ui, iead=iead)

    def sample_phase(self, bin):
        """Averages over the window's steps in one RF phase bin (n_phase bins per
        period): densities, potential, flux profiles and mean velocities."""
        n = self.nodes
        a = {k: np.zeros(n) for k in ("ne", "ni", "phi", "gamma_e", "gamma_i", "u_e", "u_i")}
        d = pm_phase_sample(**{k: _ptr(v, C.c_double) for k, v in a.items()})
        _check(pm_sample_phase(self.h, int(bin), C.byref(d), _stream(self.stream)), "pm_sample_phase")
        a.update(n_steps=d.n_steps, n_flux_samples=d.n_flux_samples, status=d.status)
        return a

    def get_particles(self, species, capacity=None):
        cap = int(capacity or (self.p["capacity_i"] if species else self.p["capacity_e"]))
        arrs = dict(xt=np.zeros(cap), ux=np.zeros(cap), uy=np.zeros(cap), uz=np.zeros(cap),
                    id=np.zeros(cap, dtype=np.uint64), next=np.zeros(cap, dtype=np.uint32))
        pp = pm_particles(n=0, capacity=cap, xt=_ptr(arrs["xt"], C.c_double), ux=_ptr(arrs["ux"], C.c_double),
                          uy=_ptr(arrs["uy"], C.c_double), uz=_ptr(arrs["uz"], C.c_double),
                          id=_ptr(arrs["id"], C.c_uint64), next=_ptr(arrs["next"], C.c_uint32))
        _check(pm_get_particles(self.h, int(species), C.byref(pp), _stream(self.stream)), "pm_get_particles")
        return {k: v[:pp.n].copy() for k, v in arrs.items()}

    def set_particles(self, species, st):
        n = int(len(st["xt"]))
        a = {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("xt", "ux", "uy", "uz")}
        ids = np.ascontiguousarray(st["id"], dtype=np.uint64)
        nx = np.ascontiguousarray(st["next"], dtype=np.uint32)
        pp = pm_particles(n=n, capacity=n, xt=_ptr(a["xt"], C.c_double), ux=_ptr(a["ux"], C.c_double),
                          uy=_ptr(a["uy"], C.c_double), uz=_ptr(a["uz"], C.c_double),
                          id=_ptr(ids, C.c_uint64), next=_ptr(nx, C.c_uint32))
        _check(pm_set_particles(self.h, int(species), C.byref(pp), _stream(self.stream)), "pm_set_particles")

    def save_checkpoint(self):
        """The case's whole state as bytes (a numpy uint8 array): see load_checkpoint."""
        buf = np.empty(int(pm_checkpoint_bytes(self.h)), dtype=np.uint8)
        _check(pm_save_checkpoint(self.h, buf.ctypes.data, buf.nbytes, _stream(self.stream)),
               "pm_save_checkpoint")
        return buf

    def load_checkpoint(self, buf):
        """Continue from a state that save_checkpoint wrote, from a case of the
        same parameters (this or another process or device)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(pm_load_checkpoint(self.h, buf.ctypes.data, buf.nbytes, _stream(self.stream)),
               "pm_load_checkpoint")

    def step_profile(self):
        """Per-workgroup timestamps (100 MHz ticks) of the last step, shape (grid, 8);
        needs PM_PROFILE=1 in the environment when the case was created."""
        g = C.c_int32()
        _check(pm_get_step_profile(self.h, None, 0, C.byref(g), _stream(self.stream)), "pm_get_step_profile")
        out = np.zeros(8 * g.value, dtype=np.uint64)
        _check(pm_get_step_profile(self.h, _ptr(out, C.c_uint64), out.size, C.byref(g), _stream(self.stream)),
               "pm_get_step_profile")
        return out.reshape(g.value, 8)

    def get_fields(self):
        n = self.nodes
        qe, qi = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
        phi, E = np.zeros(n), np.zeros(n)
        f = pm_fields(qe=_ptr(qe, C.c_int64), qi=_ptr(qi, C.c_int64), phi=_ptr(phi, C.c_double),
                      efield=_ptr(E, C.c_double))
        _check(pm_get_fields(self.h, C.byref(f), _stream(self.stream)), "pm_get_fields")
        return dict(qe=qe, qi=qi, phi=phi, E=E, sigma_init=f.sigma_init, n_absorbed_net=f.n_absorbed_net)

    def inject_sputtered(self, yield_const=1.0, table=None, u_s_ev=3.4, e_cut_ev=200.0, n_atoms=0,
                         seed=1607, job_id=3, electrode=0, since_last=False):
        """Atoms sputtered by the recorded ion impacts on one electrode; with
        since_last only the impacts since the previous since_last call (live
        coupling, ids continuing the window's atoms)."""
        te = ty = None
        sp = pm_sputter_params(yield_const=float(yield_const), n_table=0, u_s_ev=u_s_ev,
                               e_cut_ev=e_cut_ev, n_atoms=int(n_atoms), seed=int(seed), job_id=int(job_id),
                               electrode=int(electrode), since_last=int(bool(since_last)))
        if table is not None:
            te = np.ascontiguousarray(table[0], dtype=np.float64)
            ty = np.ascontiguousarray(table[1], dtype=np.float64)
            sp.n_table = te.size
            sp.table_e_ev = _ptr(te, C.c_double)
            sp.table_y = _ptr(ty, C.c_double)
        out = pm_tp_source()
        _check(pm_inject_sputtered(self.h, C.byref(sp), C.byref(out), _stream(self.stream)),
               "pm_inject_sputtered")
        return dict(n_atoms=out.n_atoms, first_atom=out.first_atom, n_impacts=out.n_impacts,
                    n_emitted=out.n_emitted, flux_m2s=out.flux_m2s, u_s_ev=out.u_s_ev,
                    e_cut_ev=out.e_cut_ev, seed=out.seed, job_id=out.job_id, electrode=out.electrode)


class Batch:
    """Independent cases advanced together in the same launches (the cases stay
    usable alone; close the batch before closing its cases)."""

    def __init__(self, cases, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("picmcc needs a GPU (no CPU path)")
        self.cases = list(cases)
        self.stream = stream
        hs = (C.c_void_p * len(self.cases))(*[c.h.value for c in self.cases])
        nbytes = pm_batch_footprint(hs, len(self.cases))
        if nbytes == 0:
            raise PicMccError(-1, "pm_batch_footprint")
        self.arena = _arena(nbytes)
        h = C.c_void_p()
        _check(pm_batch_create(hs, len(self.cases), C.c_void_p(self.arena.data_ptr()), nbytes,
                               _stream(stream), C.byref(h)), "pm_batch_create")
        self.h = h
        self._auto_work = True

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            pm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n):
        _check(pm_batch_step(self.h, int(n), _stream(self.stream)), "pm_batch_step")

    def step_rf_cycles(self, n):
        _check(pm_batch_step_rf_cycles(self.h, int(n), _stream(self.stream)), "pm_batch_step_rf_cycles")

    def time_kernels(self, n):
        """Average (push, collision) launch durations in ms over n single steps
        (lanes one after another)."""
        a, b = C.c_double(), C.c_double()
        _check(pm_batch_time_kernels(self.h, int(n), _stream(self.stream), C.byref(a), C.byref(b)),
               "pm_batch_time_kernels")
        return a.value, b.value

    def launch_shape(self):
        sh = pm_launch_shape()
        _check(pm_batch_get_launch_shape(self.h, C.byref(sh)), "pm_batch_get_launch_shape")
        return {k: getattr(sh, k) for k in SHAPE_KEYS}

    def set_launch_shape(self, **kw):
        """Change any of unroll, waves, work_groups (total), deposit_mode, sort_interval."""
        cur = self.launch_shape()
        if "work_groups" not in kw:
            kw["work_groups"] = 0 if self._auto_work else cur["work_groups"]
        self._auto_work = int(kw["work_groups"]) == 0
        cur.update(kw)
        sh = pm_launch_shape(**{k: int(cur[k]) for k in SHAPE_KEYS})
        _check(pm_batch_set_launch_shape(self.h, C.byref(sh), _stream(self.stream)), "pm_batch_set_launch_shape")

    def info(self):
        n, g = C.c_int32(), C.c_int32()
        per = (C.c_int32 * len(self.cases))()
        _check(pm_batch_info(self.h, C.byref(n), C.byref(g), per), "pm_batch_info")
        return dict(n_cases=n.value, step_workgroups=g.value, case_workgroups=list(per))


class SlotBatch(Batch):
    """A slotted batch: n_slots slots that cases join and leave between steps
    (pm_batch_set_slot) without a new graph capture."""

    def __init__(self, n_slots, steps_per_cycle, max_cells=1024, fp64=False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("picmcc needs a GPU (no CPU path)")
        self.stream = stream
        nbytes = pm_batch_slots_footprint(int(n_slots), int(bool(fp64)))
        if nbytes == 0:
            raise PicMccError(-1, "pm_batch_slots_footprint")
        self.arena = _arena(nbytes)
        h = C.c_void_p()
        _check(pm_batch_create_slots(int(n_slots), int(bool(fp64)), int(steps_per_cycle), int(max_cells),
                                     C.c_void_p(self.arena.data_ptr()), nbytes, _stream(stream), C.byref(h)),
               "pm_batch_create_slots")
        self.h = h
        self.cases = [None] * int(n_slots)
        self._auto_work = True

    def set_slot(self, slot, case):
        """Put case (a Case, or None to empty the slot) in slot."""
        _check(pm_batch_set_slot(self.h, int(slot), case.h if case is not None else None, _stream(self.stream)),
               "pm_batch_set_slot")
        self.cases[int(slot)] = case

    def info(self):
        n, g = C.c_int32(), C.c_int32()
        per = (C.c_int32 * len(self.cases))()
        _check(pm_batch_info(self.h, C.byref(n), C.byref(g), per), "pm_batch_info")
        return dict(n_cases=n.value, step_workgroups=g.value, case_workgroups=list(per))


def tp_params(tp):
    return pm_tp_params(p_pa=tp["p_pa"], t_gas_k=tp["t_gas_k"], d_ref=tp["d_ref"], omega=tp["omega"],
                        t_ref=tp["t_ref"], m_test_amu=tp["m_test_amu"], m_gas_amu=tp["m_gas_amu"],
                        gap_m=tp["gap_m"], lateral_m=tp["lateral_m"], mode=int(tp["mode"]),
                        e_max=int(tp["e_max"]), n_ebins=int(tp["n_ebins"]), ebin_ev=tp["ebin_ev"],
                        n_tbins=int(tp["n_tbins"]), tbin_s=tp["tbin_s"], n_xbins=int(tp.get("n_xbins", 0)),
                        scatter=int(tp.get("scatter", 0)), dt_s=float(tp.get("dt_s", 0.0)))


def tp_source(src):
    return pm_tp_source(n_atoms=int(src["n_atoms"]), first_atom=int(src.get("first_atom", 0)),
                        n_impacts=int(src.get("n_impacts", 0)), n_emitted=int(src.get("n_emitted", 0)),
                        flux_m2s=float(src.get("flux_m2s", 0.0)), u_s_ev=src["u_s_ev"],
                        e_cut_ev=src["e_cut_ev"], seed=int(src["seed"]), job_id=int(src["job_id"]),
                        electrode=int(src.get("electrode", 0)))


class TestParticleJob:
    """Arena and (optional) device trace buffers for repeated test-particle runs."""

    def __init__(self, tp, max_atoms=0, trace=False, stream=None):
        import torch
        self.tp = dict(tp)
        self._tpp = tp_params(self.tp)
        nbytes = pm_tp_footprint(C.byref(self._tpp))
        if nbytes == 0:
            raise PicMccError(-1, "pm_tp_footprint")
        self.nbytes = nbytes
        self.arena = _arena(nbytes)
        self.stream = stream
        self.trace_buf = None
        if trace:
            n = max(int(max_atoms), 1)
            dev = "cuda"
            self.trace_buf = dict(
                wall=torch.empty(n, dtype=torch.int32, device=dev),
                events=torch.empty(n, dtype=torch.int32, device=dev),
                **{k: torch.empty(n, dtype=torch.float32, device=dev)
                   for k in ("energy_ev", "theta_deg", "tof_s", "vx", "vy", "vz")})

    def run(self, src):
        src = dict(src)
        cs = tp_source(src)
        res, keep, tr = _tp_result(self.tp, cs.n_atoms, self.trace_buf)
        _check(pm_run_test_particles(C.byref(self._tpp), C.byref(cs), C.c_void_p(self.arena.data_ptr()),
                                     self.nbytes, _stream(self.stream), C.byref(res)), "pm_run_test_particles")
        return _tp_out(res, keep, cs.n_atoms, self.trace_buf if tr is not None else None)


def _tp_result(tp, n_atoms, trace_buf):
    """A pm_tp_result pointing at fresh host arrays (and the device trace buffers)."""
    keep = dict(e_hist=np.zeros(int(tp["n_ebins"]), dtype=np.uint64),
                theta_hist=np.zeros(TP_THETA_BINS, dtype=np.uint64),
                tof_hist=np.zeros(int(tp["n_tbins"]), dtype=np.uint64))
    res = pm_tp_result(**{k: _ptr(v, C.c_uint64) for k, v in keep.items()})
    tr = None
    if trace_buf is not None:
        if n_atoms > trace_buf["wall"].numel():
            raise ValueError("trace buffers smaller than n_atoms")
        tr = pm_tp_trace()
        for name, ctype in pm_tp_trace._fields_:
            setattr(tr, name, C.cast(C.c_void_p(trace_buf[name].data_ptr()), ctype))
        res.trace = C.pointer(tr)
        keep["_trace_struct"] = tr
    nx = int(tp.get("n_xbins", 0)) if int(tp["mode"]) == 0 else 0
    if nx:
        for k in ("time_s", "disp_m", "density_m3", "mean_vx"):
            keep[k] = np.zeros(nx)
            setattr(res, k, _ptr(keep[k], C.c_double))
    return res, keep, tr


def _tp_out(res, keep, n_atoms, trace_buf):
    out = dict(n_substrate=res.n_substrate, n_target=res.n_target, n_unfinished=res.n_unfinished,
               events=res.events, collisions=res.collisions, overflow=res.overflow,
               e_sum_substrate=res.e_sum_substrate, e_sum_target=res.e_sum_target, eta=res.eta,
               deposition_flux=res.deposition_flux, nu_max=res.nu_max, n_atoms=n_atoms,
               **{k: v for k, v in keep.items() if not k.startswith("_")})
    if trace_buf is not None:
        out["trace"] = {k: v[:n_atoms].cpu().numpy() for k, v in trace_buf.items()}
        out["trace"]["events"] = out["trace"]["events"].view(np.uint32)
    return out


def philox_words(id0, index, tag, aux, seed, stream_key, n, stream=None):
    """The generator's four output words for counters (id0 .. id0 + n - 1, index,
    tag, aux) under key (seed, stream_key), computed on the GPU: (n, 4) uint64."""
    import torch
    out = torch.empty(4 * max(int(n), 1), dtype=torch.int64, device="cuda")
    _check(pm_philox_words(C.c_uint64(int(id0) % 2 ** 64), C.c_uint64(int(index) % 2 ** 64),
                           C.c_uint64(int(tag)), C.c_uint64(int(aux)), C.c_uint64(int(seed)),
                           C.c_uint64(int(stream_key)), int(n), C.c_void_p(out.data_ptr()), _stream(stream)),
           "pm_philox_words")
    torch.cuda.synchronize()
    return out[:4 * int(n)].cpu().numpy().view(np.uint64).reshape(-1, 4)


def run_test_particles(src, tp, trace=False, stream=None):
    """Fly src['n_atoms'] sputtered atoms with flight parameters tp on the GPU."""
    job = TestParticleJob(tp, max_atoms=src["n_atoms"], trace=trace, stream=stream)
    return job.run(src)


def run_test_particles_static(src, tp, stream=None):
    """The same flight through pm_run_test_particles_static: no device arena is
    allocated, the tallies live in the library's per-GPU scratch."""
    cs = tp_source(src)
    tpp = tp_params(tp)
    res, keep, _ = _tp_result(tp, cs.n_atoms, None)
    _check(pm_run_test_particles_static(C.byref(tpp), C.byref(cs), _stream(stream), C.byref(res)),
           "pm_run_test_particles_static")
    return _tp_out(res, keep, cs.n_atoms, None)
