"""ctypes loader of libesmf.so: argument marshalling only.

The library must have been built (``python paper_2002_00322_amd/build.py`` or
``__graft_entry__.build()``); there is no fallback of any kind."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesmf.so")

ESMF_OK = 0
ESMF_ERR_INVALID_ARG = -1
ESMF_ERR_OUT_OF_MEMORY = -2
ESMF_ERR_DEVICE = -3
ESMF_ERR_NOT_SUPPORTED = -4

PREC_FP64 = 0
PREC_MIXED = 1
PREC_STORE32 = 2
STORE_FP64 = 0
STORE_FP32 = 1
STORE_DIRECT = 2   # integral-direct: no store, integrals recomputed in each build


class EsmfError(RuntimeError):
    def __init__(self, status, name, detail):
        super().__init__(f"{name}: {detail}" if detail else name)
        self.status = status


class InvalidArgument(EsmfError, ValueError):
    pass


class OutOfMemory(EsmfError, MemoryError):
    pass


class DeviceError(EsmfError):
    pass


class NotSupported(EsmfError, NotImplementedError):
    pass


_ERRS = {ESMF_ERR_INVALID_ARG: InvalidArgument, ESMF_ERR_OUT_OF_MEMORY: OutOfMemory,
         ESMF_ERR_DEVICE: DeviceError, ESMF_ERR_NOT_SUPPORTED: NotSupported}


class EriInfo(ctypes.Structure):
    _fields_ = [("nbf", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("npairs", ctypes.c_int64), ("npairs_kept", ctypes.c_int64),
                ("nquartets_kept", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("nelements_stored", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64),
                ("q_max", ctypes.c_double), ("tau", ctypes.c_double),
                ("storage", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fp64_store_bytes", ctypes.c_int64), ("workspace_bytes_plan", ctypes.c_int64 * 2)]

    def as_dict(self):
        out = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        out["workspace_bytes_plan"] = list(out["workspace_bytes_plan"])
        return out


PLAN_NAMES = {0: "two_visit", 1: "fused"}


class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("plan", ctypes.c_int32 * 16), ("occupancy", ctypes.c_int32 * 16),
                ("skip_zero", ctypes.c_int32 * 16), ("item_blocks", ctypes.c_int32 * 16),
                ("ms", ctypes.c_double * 16)]

    def as_dict(self):
        n = self.candidates
        return {"chosen": self.chosen,
                "variants": [{"plan": PLAN_NAMES.get(self.plan[i], self.plan[i]), "occupancy": self.occupancy[i],
                              "skip_zero": self.skip_zero[i], "item_blocks": self.item_blocks[i],
                              "ms": self.ms[i]} for i in range(n)]}


class BatchReport(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("units", ctypes.c_int32), ("items", ctypes.c_int32),
                ("plan", ctypes.c_int32), ("occupancy", ctypes.c_int32), ("skip_zero", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("cand_plan", ctypes.c_int32 * 16),
                ("cand_occupancy", ctypes.c_int32 * 16), ("cand_skip_zero", ctypes.c_int32 * 16),
                ("cand_ms", ctypes.c_double * 16), ("item_factor", ctypes.c_double),
                ("item_candidates", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("item_factors", ctypes.c_double * 4), ("item_ms", ctypes.c_double * 4)]

    def as_dict(self):
        return {"graph": bool(self.graph), "units": self.units, "items": self.items,
                "item_factor": self.item_factor,
                "item_tuner": [{"factor": self.item_factors[i], "ms": self.item_ms[i]}
                               for i in range(self.item_candidates)],
                "plan": PLAN_NAMES.get(self.plan, self.plan), "occupancy": self.occupancy,
                "skip_zero": self.skip_zero,
                "tuner": [{"plan": PLAN_NAMES.get(self.cand_plan[i], self.cand_plan[i]),
                           "occupancy": self.cand_occupancy[i], "skip_zero": self.cand_skip_zero[i],
                           "ms": self.cand_ms[i]} for i in range(self.candidates)]}


class ServerConfig(ctypes.Structure):
    _fields_ = [("nstreams", ctypes.c_int32), ("max_group", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("prec", ctypes.c_int),
                ("storage", ctypes.c_int), ("reserved", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("workspace_limit_bytes", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("sessions_open", ctypes.c_int32), ("sessions_rejected", ctypes.c_int32),
                ("requests_submitted", ctypes.c_int64), ("requests_completed", ctypes.c_int64),
                ("groups_launched", ctypes.c_int64), ("max_group_size", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Peaks(ctypes.Structure):
    _fields_ = [("fp64_mfma_tflops", ctypes.c_double), ("fp64_fma_tflops", ctypes.c_double),
                ("copy_tbps", ctypes.c_double), ("compute_units", ctypes.c_int32),
                ("clock_mhz", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); every symbol include/esmf.h declares
SIGNATURES = {
    "esmf_eri_prepare": (ctypes.c_int, [ctypes.c_int32, _dp, _dp, ctypes.c_double,
                                        ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "esmf_eri_prepare_cart": (ctypes.c_int, [ctypes.c_int32, _dp, _dp, _i32p, ctypes.c_double,
                                             ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "esmf_eri_prepare_contracted": (ctypes.c_int, [ctypes.c_int32, _dp, _i32p, _i32p, _dp, _dp, ctypes.c_double,
                                                   ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "esmf_eri_info_get": (ctypes.c_int, [_vp, ctypes.POINTER(EriInfo)]),
    "esmf_eri_release": (ctypes.c_int, [_vp]),
    "esmf_eri_lookup": (ctypes.c_int, [_vp, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p, _dp]),
    "esmf_fock_build": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "esmf_fock_build_sym": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "esmf_fock_build_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_vp), _i32p,
                                               ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                               ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "esmf_fock_tune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int, _vp, ctypes.POINTER(TuneReport)]),
    "esmf_fock_batched_report": (ctypes.c_int, [ctypes.POINTER(BatchReport)]),
    "esmf_fock_build_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "esmf_timing_enable": (ctypes.c_int, [ctypes.c_int32]),
    "esmf_timing_collect": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "esmf_probe_peaks": (ctypes.c_int, [ctypes.c_int64, _vp, ctypes.POINTER(Peaks)]),
    "esmf_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "esmf_server_destroy": (ctypes.c_int, [_vp]),
    "esmf_server_open_session": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, ctypes.c_double,
                                                _i32p, ctypes.POINTER(ctypes.c_int64)]),
    "esmf_server_open_session_contracted": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _i32p, _i32p, _dp, _dp,
                                                           ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                                           ctypes.POINTER(ctypes.c_int64)]),
    "esmf_server_close_session": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "esmf_server_submit": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "esmf_server_wait": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "esmf_server_stats_get": (ctypes.c_int, [_vp, ctypes.POINTER(ServerStats)]),
    "esmf_nine_densities": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                           _vp, _vp, _vp, _vp, _vp]),
    "esmf_energy_gradient": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double] + [_vp] * 11),
    "esmf_energy_two_body": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                            _vp, _vp, _vp]),
    "esmf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "esmf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libesmf.so (raises if it is missing: the HIP path is the only path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (paper_2002_00322_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status == ESMF_OK:
        return
    L = lib()
    name = L.esmf_status_string(status).decode()
    detail = L.esmf_last_error().decode()
    raise _ERRS.get(status, EsmfError)(status, name, detail)
