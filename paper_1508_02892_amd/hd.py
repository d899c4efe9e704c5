"""Thin ctypes binding of the C ABI in include/hd.h (argument marshalling only).

Every step of the discharge runs in the HIP kernels of libhd.so; this module
only converts Python parameter dicts to ``hd_params``, calls the entry points
and wraps the caller-owned output buffers as numpy arrays.  If the library is
not built, or cannot be loaded, the calls raise: there is no fallback.
PyTorch, when present, only supplies the stream the work is enqueued on.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhd.so")

HD_ABI_VERSION = 4
HD_MAX_CHANNELS = 16
STATUS = {0: "HD_OK", -1: "HD_EINVAL", -2: "HD_ENOMEM", -3: "HD_EDEVICE", -4: "HD_ECAPACITY",
          -5: "HD_ENUMERIC", -6: "HD_ESTATE", -7: "HD_ESYNC"}
KIND = {"elastic": 0, "excitation": 1, "ionization": 2, "attachment": 3}

# Every entry point declared in include/hd.h.
SYMBOLS = ["hd_abi_version", "hd_last_error", "hd_required_bytes", "hd_init_discharge",
           "hd_step", "hd_moments", "hd_get_particles", "hd_get_push_field", "hd_free",
           "hd_batch_create", "hd_batch_step", "hd_batch_moments", "hd_batch_get_particles",
           "hd_batch_free", "hd_server_create", "hd_server_submit", "hd_server_poll",
           "hd_server_stats", "hd_server_drain", "hd_server_free", "hd_profile_steps",
           "hd_diag_arith", "hd_swarm_create", "hd_swarm_run", "hd_swarm_results",
           "hd_swarm_get_ions", "hd_swarm_free", "hd_batch_get_launch", "hd_batch_set_launch",
           "hd_batch_autotune", "hd_get_launch", "hd_set_launch", "hd_autotune", "hd_grow",
           "hd_save", "hd_restore", "hd_server_cancel", "hd_batch_profile_steps",
           "hd_swarm_run_noalloc"]


class HdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class XsChannel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("product", C.c_int32), ("threshold_eV", C.c_double),
                ("sigma_m2", C.POINTER(C.c_double)), ("target_fraction", C.c_double),
                ("target_mass_amu", C.c_double)]


class IonSpecies(C.Structure):
    _fields_ = [("charge", C.c_int32), ("n_mu", C.c_int32), ("m_amu", C.c_double),
                ("en_lo_Td", C.c_double), ("en_hi_Td", C.c_double),
                ("mu_m2_Vs", C.POINTER(C.c_double)), ("init_fraction", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("precision", C.c_int32), ("ion_model", C.c_int32),
        ("n_cells", C.c_int32), ("n_energy", C.c_int32), ("n_channels", C.c_int32),
        ("sort_every", C.c_int32), ("eedf_every", C.c_int32), ("n_eedf_bins", C.c_int32),
        ("n_species", C.c_int32), ("n_macro", C.c_int64), ("capacity", C.c_int64),
        ("seed", C.c_uint64),
        ("n_gas_m3", C.c_double), ("t_gas_K", C.c_double), ("m_gas_amu", C.c_double),
        ("gap_m", C.c_double),
        ("v_amp_V", C.c_double), ("f_rf_Hz", C.c_double), ("phase_rad", C.c_double),
        ("n_e0_m3", C.c_double), ("t_e0_eV", C.c_double), ("load_lo", C.c_double),
        ("load_hi", C.c_double), ("gamma_see", C.c_double), ("e_sec_eV", C.c_double),
        ("m_ion_amu", C.c_double), ("mu_const", C.c_double), ("nu_const", C.c_double),
        ("dt_s", C.c_double), ("inv_de_per_eV", C.c_double), ("eedf_emax_eV", C.c_double),
        ("power_W_m2", C.c_double), ("power_alpha", C.c_double),
        ("channels", C.POINTER(XsChannel)), ("species", C.POINTER(IonSpecies)),
    ]


class LaunchConfig(C.Structure):
    _fields_ = [("electron_variant", C.c_int32), ("electron_groups", C.c_int32),
                ("sort_groups", C.c_int32), ("append_groups", C.c_int32),
                ("sort_tile", C.c_int32)]


def _launch_dict(c: LaunchConfig) -> dict:
    return {k: int(getattr(c, k)) for k, _ in LaunchConfig._fields_}


def _launch_struct(d: dict) -> LaunchConfig:
    c = LaunchConfig()
    for k, _ in LaunchConfig._fields_:
        setattr(c, k, int(d.get(k, 0)))
    return c


class DeviceCtx(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("device", C.c_int32), ("reserved", C.c_int32),
                ("arena", C.c_void_p), ("arena_bytes", C.c_size_t)]


_D = C.POINTER(C.c_double)


class MomentSet(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n_live", C.c_int64), ("n_slots", C.c_int64),
        ("n_nodes", C.c_int32), ("n_channels", C.c_int32), ("n_eedf_bins", C.c_int32),
        ("error", C.c_int32),
        ("n_e", _D), ("n_i", _D), ("phi", _D), ("E", _D), ("gamma_i", _D), ("n_e_avg", _D),
        ("n_i_avg", _D), ("n_species", _D), ("gamma_species", _D),
        ("cnt", C.POINTER(C.c_int64)), ("eedf_counts", C.POINTER(C.c_uint64)),
        ("eedf", _D),
        ("coll", C.c_uint64 * HD_MAX_CHANNELS), ("absorbed", C.c_uint64 * 2),
        ("emitted", C.c_uint64 * 2), ("created", C.c_uint64), ("e_overflow", C.c_uint64),
        ("see_clamped", C.c_uint64), ("n_acc", C.c_uint64), ("pushed", C.c_uint64),
        ("volt_amp", C.c_double), ("p_abs", C.c_double), ("rf_periods", C.c_int64),
        ("graph_steps", C.c_int64), ("rollbacks", C.c_int64),
    ]


class SwarmParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("precision", C.c_int32), ("n_fields", C.c_int32),
        ("n_energy", C.c_int32), ("n_ions", C.c_int64), ("seed", C.c_uint64),
        ("n_gas_m3", C.c_double), ("t_gas_K", C.c_double), ("m_ion_amu", C.c_double),
        ("m_gas_amu", C.c_double), ("t_i0_K", C.c_double), ("dt_s", C.c_double),
        ("inv_de_per_eV", C.c_double), ("rate_m3_s", _D), ("e0_V_m", _D),
    ]


class SwarmResult(C.Structure):
    _fields_ = [
        ("e0_V_m", C.c_double), ("drift_m_s", C.c_double), ("mean_energy_eV", C.c_double),
        ("mobility_m2_Vs", C.c_double), ("nu_s", C.c_double), ("collisions", C.c_uint64),
        ("overflow", C.c_uint64), ("samples", C.c_int64),
    ]


class ServerConfig(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_slots", C.c_int32), ("sort_every", C.c_int32),
                ("eedf_every", C.c_int32), ("max_cells", C.c_int32), ("max_energy", C.c_int32),
                ("max_channels", C.c_int32), ("max_eedf_bins", C.c_int32),
                ("allow_full_fluid", C.c_int32), ("reserved", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64)]


class ServerCounters(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("queued", C.c_uint64), ("running", C.c_uint64), ("intervals", C.c_uint64),
                ("particle_steps", C.c_uint64), ("bytes_in_use", C.c_uint64),
                ("busy_s", C.c_double), ("wall_s", C.c_double), ("error", C.c_int32),
                ("cancelled", C.c_int32)]


_lib = None


def lib():
    """Load libhd.so; raise if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libhd.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.hd_abi_version.restype = C.c_int32
        L.hd_last_error.restype = C.c_char_p
        L.hd_required_bytes.restype = C.c_size_t
        L.hd_required_bytes.argtypes = [C.POINTER(Params)]
        L.hd_init_discharge.argtypes = [C.POINTER(Params), C.POINTER(DeviceCtx), C.POINTER(vp)]
        L.hd_step.argtypes = [vp, C.c_int64]
        L.hd_moments.argtypes = [vp, C.POINTER(MomentSet)]
        L.hd_get_particles.argtypes = [vp] * 7 + [C.c_int64, C.POINTER(C.c_int64)]
        L.hd_get_push_field.argtypes = [vp, vp]
        L.hd_free.argtypes = [vp]
        L.hd_batch_create.argtypes = [C.POINTER(C.POINTER(Params)), C.c_int32,
                                      C.POINTER(DeviceCtx), C.POINTER(vp)]
        L.hd_batch_step.argtypes = [vp, C.c_int64]
        L.hd_batch_moments.argtypes = [vp, C.c_int32, C.POINTER(MomentSet)]
        L.hd_batch_get_particles.argtypes = [vp, C.c_int32] + [vp] * 6 + \
            [C.c_int64, C.POINTER(C.c_int64)]
        L.hd_batch_free.argtypes = [vp]
        L.hd_diag_arith.argtypes = [C.c_int32, C.c_int64, vp, vp, vp, C.POINTER(DeviceCtx)]
        L.hd_profile_steps.argtypes = [vp, C.c_int64, vp]
        L.hd_batch_profile_steps.argtypes = [vp, C.c_int64, vp]
        L.hd_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(DeviceCtx),
                                       C.POINTER(vp)]
        L.hd_server_submit.argtypes = [vp, C.POINTER(Params), C.c_int64,
                                       C.POINTER(C.c_uint64)]
        L.hd_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32),
                                     C.POINTER(MomentSet), vp]
        L.hd_server_stats.argtypes = [vp, C.POINTER(ServerCounters)]
        L.hd_server_drain.argtypes = [vp, C.c_double]
        L.hd_server_cancel.argtypes = [vp, C.c_uint64]
        L.hd_server_free.argtypes = [vp]
        L.hd_swarm_create.argtypes = [C.POINTER(SwarmParams), C.POINTER(DeviceCtx),
                                      C.POINTER(vp)]
        L.hd_swarm_run.argtypes = [vp, C.c_int64, C.c_int32]
        L.hd_swarm_results.argtypes = [vp, C.POINTER(SwarmResult)]
        L.hd_swarm_get_ions.argtypes = [vp, C.c_int32] + [vp] * 5 + [C.c_int64]
        L.hd_swarm_free.argtypes = [vp]
        L.hd_swarm_run_noalloc.argtypes = [C.POINTER(SwarmParams), C.c_int64, C.c_int64,
                                           C.POINTER(DeviceCtx), C.POINTER(SwarmResult)]
        for f in ("hd_batch_get_launch", "hd_get_launch"):
            getattr(L, f).argtypes = [vp, C.POINTER(LaunchConfig)]
        for f in ("hd_batch_set_launch", "hd_set_launch"):
            getattr(L, f).argtypes = [vp, C.POINTER(LaunchConfig)]
        L.hd_grow.argtypes = [vp, C.c_int64]
        L.hd_save.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.hd_restore.argtypes = [vp, vp, C.c_size_t]
        for f in ("hd_batch_autotune", "hd_autotune"):
            getattr(L, f).argtypes = [vp, C.c_int64, C.POINTER(LaunchConfig)]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise HdError(rc, lib().hd_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def pdtype(precision: int):
    return np.float32 if precision == 0 else np.float64


def make_params(p: dict):
    """hd_params from a parameter dict; returns (struct, keep-alive objects)."""
    chans = p.get("channels", [])
    keep = []
    arr = (XsChannel * max(1, len(chans)))()
    for k, ch in enumerate(chans):
        s = np.ascontiguousarray(ch["sigma_m2"], dtype=np.float64)
        keep.append(s)
        arr[k].kind = KIND[ch["kind"]] if isinstance(ch["kind"], str) else int(ch["kind"])
        arr[k].product = int(ch.get("product", 0))
        arr[k].threshold_eV = float(ch.get("threshold_eV", 0.0))
        arr[k].sigma_m2 = s.ctypes.data_as(_D)
        arr[k].target_fraction = float(ch.get("target_fraction", 1.0))
        arr[k].target_mass_amu = float(ch.get("target_mass_amu", 0.0))
    keep.append(arr)
    species = p.get("species", [])
    sarr = (IonSpecies * max(1, len(species)))()
    for k, q in enumerate(species):
        mu = np.ascontiguousarray(q["mu_m2_Vs"], dtype=np.float64)
        keep.append(mu)
        sarr[k].charge = int(q["charge"])
        sarr[k].n_mu = len(mu)
        sarr[k].m_amu = float(q["m_amu"])
        sarr[k].en_lo_Td = float(q["en_lo_Td"])
        sarr[k].en_hi_Td = float(q["en_hi_Td"])
        sarr[k].mu_m2_Vs = mu.ctypes.data_as(_D)
        sarr[k].init_fraction = float(q.get("init_fraction", 0.0))
    keep.append(sarr)
    P = Params()
    P.abi_version = HD_ABI_VERSION
    for name, _ in Params._fields_:
        if name in ("abi_version", "channels", "n_channels", "species", "n_species"):
            continue
        setattr(P, name, p[name])
    P.n_channels = len(chans)
    P.channels = C.cast(arr, C.POINTER(XsChannel))
    P.n_species = len(species)
    P.species = C.cast(sarr, C.POINTER(IonSpecies))
    return P, keep


def _ctx(stream=None, device=0, arena=None):
    """Device context; arena: a torch uint8 tensor on the device (its memory
    holds the handle's device state; the caller keeps it alive)."""
    c = DeviceCtx()
    if arena is not None:
        if arena.dtype.itemsize != 1 or not arena.is_contiguous() or arena.device.type != "cuda":
            raise ValueError("arena must be a contiguous byte tensor on the GPU")
        c.arena = arena.data_ptr()
        c.arena_bytes = arena.numel()
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream(device).cuda_stream
        except Exception:  # torch absent: the default stream
            stream = None
    c.stream = stream
    c.device = device
    return c


def required_bytes(p: dict) -> int:
    P, keep = make_params(p)
    return int(lib().hd_required_bytes(C.byref(P)))


class _Moments:
    def __init__(self, nn, nb, K, S=1):
        self.arrs = {k: np.zeros(nn) for k in ("n_e", "n_i", "phi", "E", "gamma_i", "n_e_avg",
                                                 "n_i_avg")}
        self.arrs["n_species"] = np.zeros(S * nn)
        self.arrs["gamma_species"] = np.zeros(S * nn)
        self.arrs["cnt"] = np.zeros(nn, np.int64)
        self.arrs["eedf_counts"] = np.zeros(nb + 1, np.uint64)
        self.arrs["eedf"] = np.zeros(nb)
        self.m = MomentSet()
        for k, a in self.arrs.items():
            setattr(self.m, k, a.ctypes.data_as(dict(MomentSet._fields_)[k]))
        self.K = K

    def result(self):
        m = self.m
        out = dict(self.arrs)
        out.update(step=m.step, n_live=m.n_live, n_slots=m.n_slots, error=m.error,
                   coll=np.array(m.coll[:self.K], np.uint64),
                   absorbed=np.array(m.absorbed[:], np.uint64),
                   emitted=np.array(m.emitted[:], np.uint64), created=int(m.created),
                   overflow=int(m.e_overflow), see_clamped=int(m.see_clamped),
                   n_acc=int(m.n_acc), pushed=int(m.pushed), volt_amp=float(m.volt_amp),
                   p_abs=float(m.p_abs), rf_periods=int(m.rf_periods),
                   graph_steps=int(m.graph_steps), rollbacks=int(m.rollbacks))
        return out


class Discharge:
    """One discharge: hd_init_discharge / hd_step / hd_moments / hd_free.
    arena: optional torch uint8 GPU tensor of at least required_bytes(params)
    that holds the discharge's device state (kept referenced here)."""

    def __init__(self, params: dict, stream=None, device: int = 0, arena=None):
        self.params = dict(params)
        self._P, self._keep = make_params(params)
        self._arena = arena
        self._ctx = _ctx(stream, device, arena)
        h = C.c_void_p()
        _check(lib().hd_init_discharge(C.byref(self._P), C.byref(self._ctx), C.byref(h)))
        self.h = h
        self.nn = params["n_cells"] + 1
        self.dt = pdtype(params["precision"])

    def step(self, n: int = 1):
        _check(lib().hd_step(self.h, int(n)))

    def moments(self) -> dict:
        M = _Moments(self.nn, self.params["n_eedf_bins"], len(self.params["channels"]),
                     max(1, len(self.params.get("species", []))))
        _check(lib().hd_moments(self.h, C.byref(M.m)))
        return M.result()

    def particles(self) -> dict:
        n = C.c_int64()
        cap = int(self.params["capacity"]) + 8192
        out = {"cell": np.empty(cap, np.int32), "id": np.empty(cap, np.uint32)}
        for k in ("off", "vx", "vy", "vz"):
            out[k] = np.empty(cap, self.dt)
        _check(lib().hd_get_particles(self.h, _ptr(out["cell"]), _ptr(out["off"]),
                                      _ptr(out["vx"]), _ptr(out["vy"]), _ptr(out["vz"]),
                                      _ptr(out["id"]), cap, C.byref(n)))
        return {k: v[:n.value].copy() for k, v in out.items()}

    def push_field(self) -> np.ndarray:
        ep = np.empty(self.nn, self.dt)
        _check(lib().hd_get_push_field(self.h, _ptr(ep)))
        return ep

    def grow(self, new_capacity: int):
        """Raise the particle capacity (continues a run rolled back at an overflow)."""
        _check(lib().hd_grow(self.h, int(new_capacity)))
        self.params["capacity"] = int(new_capacity)

    def save(self) -> bytes:
        """Snapshot of the run at its current step (for resume)."""
        n = C.c_size_t(0)
        _check(lib().hd_save(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().hd_save(self.h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def restore(self, snapshot: bytes):
        """Continue from a snapshot taken from a discharge of the same parameters."""
        _check(lib().hd_restore(self.h, snapshot, len(snapshot)))

    def get_launch(self) -> dict:
        c = LaunchConfig()
        _check(lib().hd_get_launch(self.h, C.byref(c)))
        return _launch_dict(c)

    def set_launch(self, cfg: dict):
        _check(lib().hd_set_launch(self.h, C.byref(_launch_struct(cfg))))

    def autotune(self, max_steps: int = 128) -> dict:
        c = LaunchConfig()
        _check(lib().hd_autotune(self.h, int(max_steps), C.byref(c)))
        return _launch_dict(c)

    def profile_steps(self, n: int) -> dict:
        """Advance n real steps with per-kernel HIP events; mean ms per kernel."""
        out = np.zeros(5)
        _check(lib().hd_profile_steps(self.h, int(n), _ptr(out)))
        return dict(zip(["electron", "finalize_field", "append", "sort", "step"], out.tolist()))

    def close(self):
        if getattr(self, "h", None):
            lib().hd_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent discharges advanced together: hd_batch_*."""

    def __init__(self, params_list, stream=None, device: int = 0, arena=None):
        self.params = [dict(p) for p in params_list]
        made = [make_params(p) for p in params_list]
        self._keep = made
        arr = (C.POINTER(Params) * len(made))(*[C.pointer(m[0]) for m in made])
        self._arr = arr
        self._arena = arena
        self._ctx = _ctx(stream, device, arena)
        h = C.c_void_p()
        _check(lib().hd_batch_create(arr, len(made), C.byref(self._ctx), C.byref(h)))
        self.h = h

    def step(self, n: int = 1):
        _check(lib().hd_batch_step(self.h, int(n)))

    def get_launch(self) -> dict:
        c = LaunchConfig()
        _check(lib().hd_batch_get_launch(self.h, C.byref(c)))
        return _launch_dict(c)

    def set_launch(self, cfg: dict):
        _check(lib().hd_batch_set_launch(self.h, C.byref(_launch_struct(cfg))))

    def autotune(self, max_steps: int = 128) -> dict:
        c = LaunchConfig()
        _check(lib().hd_batch_autotune(self.h, int(max_steps), C.byref(c)))
        return _launch_dict(c)

    def profile_steps(self, n: int) -> dict:
        """Advance n real steps with per-kernel HIP events; mean ms per kernel."""
        out = np.zeros(5)
        _check(lib().hd_batch_profile_steps(self.h, int(n), _ptr(out)))
        return dict(zip(["electron", "finalize_field", "append", "sort", "step"], out.tolist()))

    def moments(self, i: int) -> dict:
        p = self.params[i]
        M = _Moments(p["n_cells"] + 1, p["n_eedf_bins"], len(p["channels"]),
                     max(1, len(p.get("species", []))))
        _check(lib().hd_batch_moments(self.h, int(i), C.byref(M.m)))
        return M.result()

    def particles(self, i: int) -> dict:
        p = self.params[i]
        dt = pdtype(p["precision"])
        cap = int(p["capacity"]) + 8192
        n = C.c_int64()
        out = {"cell": np.empty(cap, np.int32), "id": np.empty(cap, np.uint32)}
        for k in ("off", "vx", "vy", "vz"):
            out[k] = np.empty(cap, dt)
        _check(lib().hd_batch_get_particles(self.h, int(i), _ptr(out["cell"]), _ptr(out["off"]),
                                            _ptr(out["vx"]), _ptr(out["vy"]), _ptr(out["vz"]),
                                            _ptr(out["id"]), cap, C.byref(n)))
        return {k: v[:n.value].copy() for k, v in out.items()}

    def close(self):
        if getattr(self, "h", None):
            lib().hd_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Served job stream: hd_server_create / submit / poll / stats / drain / free."""

    def __init__(self, precision=0, max_slots=64, sort_every=16, eedf_every=16, max_cells=4096,
                 max_energy=4096, max_channels=3, max_eedf_bins=128, allow_full_fluid=False,
                 hbm_budget_bytes=200 * 10 ** 9, stream=None, device=0):
        cfg = ServerConfig(precision, max_slots, sort_every, eedf_every, max_cells, max_energy,
                           max_channels, max_eedf_bins, int(allow_full_fluid), 0,
                           int(hbm_budget_bytes))
        self._ctx = _ctx(stream, device)
        h = C.c_void_p()
        _check(lib().hd_server_create(C.byref(cfg), C.byref(self._ctx), C.byref(h)))
        self.h = h
        self.jobs = {}

    def submit(self, params: dict, n_steps: int) -> int:
        P, keep = make_params(params)
        jid = C.c_uint64()
        _check(lib().hd_server_submit(self.h, C.byref(P), int(n_steps), C.byref(jid)))
        self.jobs[jid.value] = dict(params)
        return jid.value

    def poll(self, job_id: int):
        """(state, times[3], moments or None); state 0 queued, 1 running, 2 done, 3 failed,
        4 cancelled."""
        p = self.jobs[job_id]
        M = _Moments(p["n_cells"] + 1, p["n_eedf_bins"], len(p["channels"]),
                     max(1, len(p.get("species", []))))
        st = C.c_int32()
        t = np.zeros(3)
        _check(lib().hd_server_poll(self.h, C.c_uint64(job_id), C.byref(st), C.byref(M.m),
                                    _ptr(t)))
        return st.value, t, (M.result() if st.value == 2 else None)

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().hd_server_stats(self.h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def cancel(self, job_id: int):
        """Cancel a queued or running job (state 4, no result)."""
        _check(lib().hd_server_cancel(self.h, int(job_id)))

    def drain(self, timeout_s: float = 600.0):
        _check(lib().hd_server_drain(self.h, float(timeout_s)))

    def close(self):
        if getattr(self, "h", None):
            lib().hd_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diag_arith(precision: int, a, b) -> np.ndarray:
    """Device sqrt, divide, rint(x 2^32) and floor of the inputs (n x 4)."""
    dt = pdtype(precision)
    a = np.ascontiguousarray(a, dt)
    b = np.ascontiguousarray(b, dt)
    out = np.empty((len(a), 4), dt)
    ctx = _ctx()
    _check(lib().hd_diag_arith(precision, len(a), _ptr(a), _ptr(b), _ptr(out), C.byref(ctx)))
    return out


def _swarm_params(params: dict):
    """hd_swarm_params and the arrays it points into (keep them alive)."""
    rate = np.ascontiguousarray(params["rate_m3_s"], np.float64)
    e0 = np.ascontiguousarray(params["e0_V_m"], np.float64)
    P = SwarmParams()
    P.abi_version = HD_ABI_VERSION
    for name, _ in SwarmParams._fields_:
        if name in ("abi_version", "rate_m3_s", "e0_V_m", "n_energy", "n_fields"):
            continue
        setattr(P, name, params[name])
    P.n_energy = len(rate)
    P.n_fields = len(e0)
    P.rate_m3_s = rate.ctypes.data_as(_D)
    P.e0_V_m = e0.ctypes.data_as(_D)
    return P, rate, e0


def swarm_run_noalloc(params: dict, n_relax: int, n_avg: int, stream=None, device: int = 0):
    """hd_swarm_run_noalloc: the swarm in one call without device allocation."""
    P, rate, e0 = _swarm_params(params)
    ctx = _ctx(stream, device)
    out = (SwarmResult * len(e0))()
    _check(lib().hd_swarm_run_noalloc(C.byref(P), int(n_relax), int(n_avg), C.byref(ctx), out))
    del rate, e0  # kept alive until the call returned
    return [{k: getattr(r, k) for k, _ in SwarmResult._fields_} for r in out]


class Swarm:
    """Auxiliary ion swarms (one per field value): hd_swarm_create / run /
    results / get_ions / free."""

    def __init__(self, params: dict, stream=None, device: int = 0):
        self.params = dict(params)
        P, self._rate, self._e0 = _swarm_params(params)
        self._P = P
        self._ctx = _ctx(stream, device)
        h = C.c_void_p()
        _check(lib().hd_swarm_create(C.byref(P), C.byref(self._ctx), C.byref(h)))
        self.h = h
        self.n = int(params["n_ions"])
        self.D = len(self._e0)
        self.dt = pdtype(params["precision"])

    def run(self, n: int, accumulate: bool = False):
        _check(lib().hd_swarm_run(self.h, int(n), int(bool(accumulate))))

    def results(self) -> list:
        out = (SwarmResult * self.D)()
        _check(lib().hd_swarm_results(self.h, out))
        return [{k: getattr(r, k) for k, _ in SwarmResult._fields_} for r in out]

    def ions(self, f: int) -> dict:
        o = {k: np.empty(self.n, self.dt) for k in ("vx", "vy", "vz")}
        o["acc_vz"] = np.empty(self.n)
        o["acc_v2"] = np.empty(self.n)
        _check(lib().hd_swarm_get_ions(self.h, int(f), *[_ptr(o[k]) for k in
                                                          ("vx", "vy", "vz", "acc_vz", "acc_v2")],
                                       self.n))
        return o

    def close(self):
        if getattr(self, "h", None):
            lib().hd_swarm_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
