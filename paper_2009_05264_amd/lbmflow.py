"""ctypes binding of liblbmflow.so (C ABI in include/lbmflow.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of the library.  PyTorch, when used, supplies device memory
(``data_ptr``) and streams; nothing here computes physics.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmflow.so")

LBM_OK = 0
LBM_E_INVALID, LBM_E_NOMEM, LBM_E_CAP, LBM_E_DEVICE, LBM_E_NAN, LBM_E_STATE = -1, -2, -3, -4, -5, -6
STORE_F32, STORE_F32_DEV, STORE_F16_DEV, STORE_BF16_DEV = 0, 1, 2, 3
BCX_PERIODIC, BCX_CHANNEL, BCX_CHANNEL_P = 0, 1, 2
BCY_PERIODIC, BCY_WALLS = 0, 1
SIDE_S, SIDE_N = 0, 1
NOALLOC_MAX_NODES = 1 << 20  # LBM_NOALLOC_MAX_NODES


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbmflow error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "nx", "ny", "storage", "bc_x", "bc_y", "isothermal", "single_phase", "reserved")] + [
        (n, C.c_double) for n in (
            "a", "b", "R", "omega", "beta", "c0", "g", "tau_f", "s_e", "s_eps", "s_q",
            "tau_g", "c_v", "ga_x", "ga_y", "fb_x", "fb_y", "u_in", "T_in", "U_out",
            "T_iso", "rho_mid", "rho_ref", "T_ref", "rho_out", "G_wet")]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64)] + [(n, C.c_double) for n in (
        "mass", "energy", "heater_q", "vapor_cells", "psi_clamped", "nonfinite", "p_in", "p_out", "nu_heater",
        "dp")]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class Request(C.Structure):
    _fields_ = [("T_wall_s", C.POINTER(C.c_double)), ("rho_w_s", C.POINTER(C.c_double)),
                ("heater", C.POINTER(C.c_int32)), ("T_wall_n", C.POINTER(C.c_double)),
                ("rho_w_n", C.POINTER(C.c_double)), ("rho_init", C.c_double), ("T_init", C.c_double),
                ("noise", C.c_double), ("seed", C.c_uint64)]


class ServerInfo(C.Structure):
    _fields_ = [("queued", C.c_int64), ("running", C.c_int64), ("done", C.c_int64),
                ("resident_bytes", C.c_size_t), ("peak_resident_bytes", C.c_size_t),
                ("lups", C.c_double), ("busy_seconds", C.c_double), ("failed", C.c_int64)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, 4

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp, dp, fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float)
        sig = {
            "lbm_last_error": (C.c_char_p, []),
            "lbm_params_default": (C.c_int, [C.POINTER(Params)]),
            "lbm_neutral_G_wet": (C.c_double, [C.POINTER(Params)]),
            "lbm_required_bytes": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
            "lbm_create": (C.c_int, [C.POINTER(Params), vp, vp, C.c_size_t, C.POINTER(vp)]),
            "lbm_destroy": (C.c_int, [vp]),
            "lbm_set_wall_maps": (C.c_int, [vp, C.c_int, dp, dp, C.POINTER(C.c_int32)]),
            "lbm_init_fields": (C.c_int, [vp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_uint64]),
            "lbm_init_fields_noalloc": (C.c_int, [vp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_uint64]),
            "lbm_step": (C.c_int, [vp, C.c_int64]),
            "lbm_sync": (C.c_int, [vp]),
            "lbm_step_count": (C.c_int64, [vp]),
            "lbm_read_fields": (C.c_int, [vp, dp, dp, dp, dp]),
            "lbm_read_fields_device": (C.c_int, [vp, vp, vp, vp, vp]),
            "lbm_read_diag": (C.c_int, [vp, C.POINTER(Diag)]),
            "lbm_diag_history": (C.c_int, [vp, C.POINTER(Diag), C.c_int, C.POINTER(C.c_int)]),
            "lbm_save": (C.c_int, [vp, C.c_char_p]),
            "lbm_load": (C.c_int, [vp, C.c_char_p]),
            "lbm_maxwell": (C.c_int, [C.POINTER(Params), C.c_double, dp, dp, dp]),
            "lbm_set_tile_rows": (C.c_int, [vp, C.c_int]),
            "lbm_tile_plan": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                                        C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int,
                                        C.POINTER(C.c_int)]),
            "lbm_batch_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_char_p, C.POINTER(vp)]),
            "lbm_batch_step": (C.c_int, [vp, C.c_int64]),
            "lbm_batch_sync": (C.c_int, [vp]),
            "lbm_batch_destroy": (C.c_int, [vp]),
            "lbm_stream_copy": (C.c_int, [vp, vp, C.c_size_t, vp]),
            "lbm_server_create": (C.c_int, [C.c_size_t, C.c_int, C.c_int64, vp, C.POINTER(vp)]),
            "lbm_server_submit": (C.c_int, [vp, C.POINTER(Params), C.POINTER(Request), C.c_int64,
                                            C.POINTER(C.c_uint64)]),
            "lbm_server_pump": (C.c_int, [vp, C.POINTER(C.c_int)]),
            "lbm_server_pump_async": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "lbm_server_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(C.c_int), dp]),
            "lbm_server_read_fields": (C.c_int, [vp, C.c_uint64, dp, dp, dp, dp]),
            "lbm_server_read_diag": (C.c_int, [vp, C.c_uint64, C.POINTER(Diag)]),
            "lbm_server_release": (C.c_int, [vp, C.c_uint64]),
            "lbm_server_cancel": (C.c_int, [vp, C.c_uint64]),
            "lbm_server_stats": (C.c_int, [vp, C.POINTER(ServerInfo)]),
            "lbm_server_destroy": (C.c_int, [vp]),
            "lbm_admission_plan": (C.c_int, [C.POINTER(C.c_size_t), C.c_int, C.c_size_t, C.c_size_t,
                                             C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_params(**kw) -> Params:
    """lbm_params_default with the given fields replaced; G_wet, when not
    given (or None), is the library's neutral value for the final beta and g."""
    p = Params()
    _check(lib().lbm_params_default(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        if v is not None:
            setattr(p, k, v)
    if kw.get("G_wet") is None:
        p.G_wet = lib().lbm_neutral_G_wet(C.byref(p))
    return p


def required_bytes(p: Params) -> int:
    n = C.c_size_t()
    _check(lib().lbm_required_bytes(C.byref(p), C.byref(n)))
    return n.value


def maxwell(p: Params, T: float):
    rl, rv, ps = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_maxwell(C.byref(p), float(T), C.byref(rl), C.byref(rv), C.byref(ps)))
    return rl.value, rv.value, ps.value


def tile_plan(nx: int, ny: int, storage: int = 1, simds: int = 0, rows: int = 0):
    """The tiling lbm_create makes (host only): (rows per tile, [(x0, y0, y1), ...])."""
    n, r = C.c_int(), C.c_int()
    _check(lib().lbm_tile_plan(nx, ny, storage, simds, rows, C.byref(r), None, None, None, 0, C.byref(n)))
    a = [(C.c_int * max(n.value, 1))() for _ in range(3)]
    _check(lib().lbm_tile_plan(nx, ny, storage, simds, rows, C.byref(r), a[0], a[1], a[2], n.value, C.byref(n)))
    return r.value, [(a[0][i], a[1][i], a[2][i]) for i in range(n.value)]


def stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int | None = None):
    _check(lib().lbm_stream_copy(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes, C.c_void_p(stream or 0)))


class Domain:
    """One channel/box domain on the current HIP device."""

    def __init__(self, params: Params, stream: int | None = None, device_buffer=None):
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        h = C.c_void_p()
        ptr, nbytes = None, 0
        self._buf = device_buffer  # keep the caller's tensor alive
        if device_buffer is not None:
            ptr = C.c_void_p(device_buffer.data_ptr())
            nbytes = device_buffer.numel() * device_buffer.element_size()
        _check(lib().lbm_create(C.byref(params), C.c_void_p(stream or 0), ptr, nbytes, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().lbm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_wall(self, side: int, T_wall, rho_w, heater=None):
        Tw = np.ascontiguousarray(np.broadcast_to(np.asarray(T_wall, float), (self.nx,)))
        rw = np.ascontiguousarray(np.broadcast_to(np.asarray(rho_w, float), (self.nx,)))
        hp = None
        if heater is not None:
            ha = np.ascontiguousarray(np.asarray(heater, dtype=np.int32))
            hp = ha.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().lbm_set_wall_maps(self.h, int(side), _dp(Tw), _dp(rw), hp))

    def init(self, rho0=None, T0=None, rho_u=1.0, T_u=None, noise=0.0, seed=0):
        T_u = self.params.T_in if T_u is None else T_u
        shp = (self.ny, self.nx)
        r = None if rho0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(rho0, float), shp))
        t = None if T0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(T0, float), shp))
        _check(lib().lbm_init_fields(self.h, None if r is None else _dp(r), None if t is None else _dp(t),
                                     float(rho_u), float(T_u), float(noise), C.c_uint64(seed)))

    def step(self, n: int = 1):
        _check(lib().lbm_step(self.h, int(n)))

    def sync(self):
        _check(lib().lbm_sync(self.h))

    @property
    def steps(self) -> int:
        return int(lib().lbm_step_count(self.h))

    def fields(self) -> dict:
        shp = (self.ny, self.nx)
        out = {k: np.zeros(shp) for k in ("rho", "ux", "uy", "T")}
        _check(lib().lbm_read_fields(self.h, *[_dp(out[k]) for k in ("rho", "ux", "uy", "T")]))
        return out

    def fields_device(self, rho, ux, uy, T):
        """Write the fields into caller device buffers (e.g. torch float32 tensors)."""
        ptrs = [C.c_void_p(t.data_ptr()) if t is not None else None for t in (rho, ux, uy, T)]
        _check(lib().lbm_read_fields_device(self.h, *ptrs))

    def diag(self) -> dict:
        d = Diag()
        _check(lib().lbm_read_diag(self.h, C.byref(d)))
        return d.as_dict()

    def diag_history(self, max_records: int = 4096) -> list:
        arr = (Diag * max_records)()
        n = C.c_int()
        _check(lib().lbm_diag_history(self.h, arr, max_records, C.byref(n)))
        return [arr[i].as_dict() for i in range(n.value)]

    def save(self, path: str):
        _check(lib().lbm_save(self.h, path.encode()))

    def load(self, path: str):
        _check(lib().lbm_load(self.h, path.encode()))

    def set_tile_rows(self, rows: int):
        _check(lib().lbm_set_tile_rows(self.h, int(rows)))


class Batch:
    """Several initialised domains stepped together, one launch per step."""

    def __init__(self, domains, tune_cache: str | None = None):
        self.domains = list(domains)
        arr = (C.c_void_p * len(self.domains))(*[d.h.value for d in self.domains])
        h = C.c_void_p()
        _check(lib().lbm_batch_create(arr, len(self.domains),
                                      None if tune_cache is None else tune_cache.encode(), C.byref(h)))
        self.h = h

    def step(self, n: int):
        _check(lib().lbm_batch_step(self.h, int(n)))

    def sync(self):
        _check(lib().lbm_batch_sync(self.h))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().lbm_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def admission_plan(footprints, cap: int, used: int, free_slots: int) -> list:
    """The server's admission rule (host only): indices admitted in order."""
    n = len(footprints)
    fp = (C.c_size_t * max(n, 1))(*[int(f) for f in footprints])
    adm = (C.c_int * max(n, 1))()
    na = C.c_int()
    _check(lib().lbm_admission_plan(fp, n, int(cap), int(used), int(free_slots), adm, C.byref(na)))
    return [adm[i] for i in range(na.value)]


class Server:
    """Continuous-batching server of flow-boiling solves (lbm_server_*)."""

    def __init__(self, cap_bytes: int, max_slots: int = 256, quantum: int = 500, stream: int | None = None):
        h = C.c_void_p()
        _check(lib().lbm_server_create(int(cap_bytes), int(max_slots), int(quantum), C.c_void_p(stream or 0),
                                       C.byref(h)))
        self.h = h

    def submit(self, params: Params, budget: int, walls=None, rho_init=1.0, T_init=1.0, noise=0.0,
               seed=0) -> int:
        """walls: (T_south, rho_w_south, heater, T_north, rho_w_north), each [nx] (heater may be None)."""
        r = Request()
        keep = []
        if walls is not None:
            Ts, rws, heat, Tn, rwn = walls
            arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, float), (params.nx,)))
                    for a in (Ts, rws, Tn, rwn)]
            keep += arrs
            r.T_wall_s, r.rho_w_s, r.T_wall_n, r.rho_w_n = [_dp(a) for a in arrs]
            if heat is not None:
                ha = np.ascontiguousarray(np.asarray(heat, dtype=np.int32))
                keep.append(ha)
                r.heater = ha.ctypes.data_as(C.POINTER(C.c_int32))
        r.rho_init, r.T_init, r.noise, r.seed = float(rho_init), float(T_init), float(noise), int(seed)
        rid = C.c_uint64()
        _check(lib().lbm_server_submit(self.h, C.byref(params), C.byref(r), int(budget), C.byref(rid)))
        return rid.value

    def pump(self) -> int:
        n = C.c_int()
        _check(lib().lbm_server_pump(self.h, C.byref(n)))
        return n.value

    def pump_async(self) -> tuple[int, bool]:
        """Non-blocking round: (requests running, a quantum is on the device)."""
        n, f = C.c_int(), C.c_int()
        _check(lib().lbm_server_pump_async(self.h, C.byref(n), C.byref(f)))
        return n.value, bool(f.value)

    def poll(self, rid: int):
        st, t = C.c_int(), C.c_double()
        _check(lib().lbm_server_poll(self.h, rid, C.byref(st), C.byref(t)))
        return st.value, t.value

    def fields(self, rid: int, nx: int, ny: int) -> dict:
        out = {k: np.zeros((ny, nx)) for k in ("rho", "ux", "uy", "T")}
        _check(lib().lbm_server_read_fields(self.h, rid, *[_dp(out[k]) for k in ("rho", "ux", "uy", "T")]))
        return out

    def diag(self, rid: int) -> dict:
        d = Diag()
        _check(lib().lbm_server_read_diag(self.h, rid, C.byref(d)))
        return d.as_dict()

    def release(self, rid: int):
        _check(lib().lbm_server_release(self.h, rid))

    def cancel(self, rid: int):
        _check(lib().lbm_server_cancel(self.h, rid))

    def stats(self) -> dict:
        s = ServerInfo()
        _check(lib().lbm_server_stats(self.h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().lbm_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
