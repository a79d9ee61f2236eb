"""Thin ctypes binding of libcamelot (include/camelot.h): argument marshalling only.

Every computation runs in the library (HIP kernels on the GPU, C++ on the host for
the allocator). Importing this module raises if libcamelot.so has not been built;
there is no fallback path. Device buffers are passed as integers (e.g. a torch
tensor's ``data_ptr()``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcamelot.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_02088_amd.build`")
_lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

# ------------------------------------------------------------------ constants
OK, EINVAL, ENOMEM, EAGAIN, ETIMEDOUT, EINFEASIBLE, EDEVICE, ESTOPPED = 0, -1, -2, -3, -4, -5, -6, -7
MAX_STAGES, MAX_LAYERS, MAX_K, MAX_BATCH = 8, 8, 128, 128
NOALLOC_SCRATCH_BYTES = 8 << 20          # CAMELOT_NOALLOC_SCRATCH_BYTES
(STAGE_GEMM_RELU, STAGE_GEMM_ARGMAX, STAGE_LOGMEL, STAGE_MLP_BF16, STAGE_TOPK, STAGE_GATHER, STAGE_CONV_POOL,
 STAGE_GATHER_SCORE, STAGE_ARTIFACT_P, STAGE_ARTIFACT_C, STAGE_ARTIFACT_M) = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11
HANDOFF_DEVICE, HANDOFF_HOST = 0, 1
INGEST_HOST, INGEST_REPLAY, INGEST_IPC = 0, 1, 2
IPC_HANDLE_BYTES = 64
IPC_PRODUCER, IPC_CONSUMER = 0, 1
PRED_NIN, PRED_NHID = 16, 64
PRED_NPARAMS = 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1

_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EAGAIN: "EAGAIN", ETIMEDOUT: "ETIMEDOUT",
          EINFEASIBLE: "EINFEASIBLE", EDEVICE: "EDEVICE", ESTOPPED: "ESTOPPED"}


class CamelotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


# ------------------------------------------------------------------ structs
class DeviceInfo(C.Structure):
    _fields_ = [("n_cus", C.c_int32), ("n_xcds", C.c_int32), ("wall_clock_hz", C.c_int64),
                ("hbm_bytes", C.c_int64), ("arch", C.c_char * 32)]


class Problem(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("cu_total", C.c_int32), ("cu_step", C.c_int32),
                ("max_instances", C.c_int32), ("max_inst_per_stage", C.c_int32),
                ("n_batches", C.c_int32), ("batches", C.POINTER(C.c_int32)),
                ("qos_ns", C.c_int64), ("hbm_bytes_budget", C.c_int64), ("hbm_bw_budget", C.c_int64),
                ("lat_ns", C.POINTER(C.c_int64)), ("bw_bps", C.POINTER(C.c_int64)),
                ("mem_bytes", C.POINTER(C.c_int64)), ("batch_wait_ns", C.POINTER(C.c_int64)),
                ("inst_max", C.POINTER(C.c_int32))]


class Alloc(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("batch", C.c_int32), ("batch_index", C.c_int32),
                ("n", C.c_int32 * MAX_STAGES), ("cu", C.c_int32 * MAX_STAGES),
                ("thr_num", C.c_int64), ("thr_den", C.c_int64), ("lat_ns", C.c_int64),
                ("cu_used", C.c_int64)]

    def as_dict(self):
        S = self.n_stages
        return {"batch": self.batch, "batch_index": self.batch_index, "n": list(self.n[:S]),
                "cu": list(self.cu[:S]), "thr_num": self.thr_num, "thr_den": self.thr_den,
                "lat_ns": self.lat_ns, "cu_used": self.cu_used}


class StageDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_layers", C.c_int32), ("dims", C.c_int32 * (MAX_LAYERS + 1)),
                ("k", C.c_int32), ("weights", C.c_void_p * MAX_LAYERS)]


class PipelineConfig(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("stages", StageDesc * MAX_STAGES), ("cu", C.c_int32 * MAX_STAGES),
                ("n_inst", C.c_int32 * MAX_STAGES), ("cu_offset", C.c_int32), ("max_batch", C.c_int32), ("batch_target", C.c_int32),
                ("batch_timeout_ns", C.c_int64), ("ring_depth", C.c_int32), ("handoff", C.c_int32),
                ("ingest", C.c_int32), ("max_rows_per_request", C.c_int32), ("ingest_capacity", C.c_int32),
                ("egress_capacity", C.c_int32), ("idle_timeout_ns", C.c_int64),
                ("hbm_budget_bytes", C.c_int64), ("side_bytes", C.c_int32), ("out_ipc", C.c_int32),
                ("ipc_handle", C.c_uint8 * IPC_HANDLE_BYTES)]


class Result(C.Structure):
    _fields_ = [("query_id", C.c_uint64), ("row", C.c_int32), ("n_out", C.c_int32),
                ("idx", C.c_int32 * MAX_K), ("val", C.c_float * MAX_K),
                ("t_ns", C.c_uint64 * (2 * MAX_STAGES + 2))]


class PipelineStats(C.Structure):
    _fields_ = [("submitted_requests", C.c_uint64), ("submitted_rows", C.c_uint64),
                ("delivered_rows", C.c_uint64), ("batches", C.c_uint64 * MAX_STAGES),
                ("id_sum", C.c_uint64 * MAX_STAGES), ("id_xor", C.c_uint64 * MAX_STAGES),
                ("worker_status", C.c_int32 * MAX_STAGES),
                ("rows", C.c_uint64 * MAX_STAGES), ("busy_ns", C.c_int64 * MAX_STAGES),
                ("wait_ns", C.c_int64 * MAX_STAGES)]


MAX_CORUN = 8


class CorunRecord(C.Structure):
    _fields_ = [("m", C.c_int32), ("kinds", C.c_int32 * MAX_CORUN), ("cu", C.c_int32 * MAX_CORUN),
                ("bi", C.c_int32 * MAX_CORUN), ("ns", C.c_double * MAX_CORUN)]


class SoloTables(C.Structure):
    _fields_ = [("n_kinds", C.c_int32), ("cu_step", C.c_int32), ("n_shares", C.c_int32),
                ("n_batches", C.c_int32), ("batches", C.POINTER(C.c_int32)), ("hbm", C.POINTER(C.c_float)),
                ("mfma", C.POINTER(C.c_float))]


STRUCTS = {"camelot_corun_record": CorunRecord, "camelot_solo_tables": SoloTables,
           "camelot_device_info": DeviceInfo, "camelot_problem": Problem, "camelot_alloc": Alloc,
           "camelot_stage_desc": StageDesc, "camelot_pipeline_config": PipelineConfig,
           "camelot_result": Result, "camelot_pipeline_stats": PipelineStats}

# ------------------------------------------------------------------ prototypes
_P = C.c_void_p
_SIGS = {
    "camelot_last_error": (C.c_char_p, []),
    "camelot_version": (C.c_int32, []),
    "camelot_device_query": (C.c_int32, [C.POINTER(DeviceInfo)]),
    "camelot_alloc_peak": (C.c_int32, [C.POINTER(Problem), C.POINTER(Alloc)]),
    "camelot_alloc_min": (C.c_int32, [C.POINTER(Problem), C.c_int64, C.c_int64, C.POINTER(Alloc)]),
    "camelot_alloc_eval": (C.c_int32, [C.POINTER(Problem), C.POINTER(Alloc)]),
    "camelot_stage_row_bytes_in": (C.c_int64, [C.POINTER(StageDesc)]),
    "camelot_stage_row_bytes_out": (C.c_int64, [C.POINTER(StageDesc)]),
    "camelot_stage_run": (C.c_int32, [C.POINTER(StageDesc), _P, _P, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "camelot_stage_run_noalloc": (C.c_int32, [C.POINTER(StageDesc), _P, _P, C.c_int32, C.c_int32, C.c_int32,
                                              _P]),
    "camelot_stream_bench": (C.c_int32, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_double)]),
    "camelot_pipeline_submit_replay": (C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P, C.c_int64]),
    "camelot_pipeline_submit_status": (C.c_int32, [_P, C.POINTER(C.c_int64)]),
    "camelot_alloc_sa": (C.c_int32, [C.POINTER(Problem), C.c_int32, C.c_int64, C.c_int64, C.c_int32, C.c_uint64,
                                     C.POINTER(Alloc)]),
    "camelot_pipeline_create": (C.c_int32, [C.POINTER(PipelineConfig), C.POINTER(_P)]),
    "camelot_pipeline_footprint": (C.c_int64, [_P]),
    "camelot_pipeline_epoch_ns": (C.c_int32, [_P, C.POINTER(C.c_int64)]),
    "camelot_pipeline_submit": (C.c_int32, [_P, C.c_uint64, _P, C.c_int32]),
    "camelot_pipeline_drain": (C.c_int32, [_P, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32),
                                           C.c_int64]),
    "camelot_pipeline_drain_latency": (C.c_int32, [_P, _P, _P, C.c_int32, C.POINTER(C.c_int32), C.c_int64]),
    "camelot_pipeline_replay": (C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P, C.c_int64]),
    "camelot_pipeline_stats_get": (C.c_int32, [_P, C.POINTER(PipelineStats)]),
    "camelot_pipeline_destroy": (C.c_int32, [_P, C.POINTER(C.c_uint64)]),
    "camelot_server_create": (C.c_int32, [C.c_int64, C.POINTER(_P)]),
    "camelot_server_admit": (C.c_int32, [_P, C.POINTER(PipelineConfig), C.POINTER(_P)]),
    "camelot_server_release": (C.c_int32, [_P, _P, C.POINTER(C.c_uint64)]),
    "camelot_server_used_bytes": (C.c_int64, [_P]),
    "camelot_server_destroy": (C.c_int32, [_P]),
    "camelot_stage_weight_bytes": (C.c_int64, [C.POINTER(StageDesc)]),
    "camelot_stage_kernel_info": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int32)]),
    "camelot_handoff_bench": (C.c_int32, [C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_int32,
                                          C.c_int32, C.POINTER(C.c_double)]),
    "camelot_handoff_expected": (C.c_int32, [C.c_int64, C.c_int64, C.POINTER(C.c_uint64),
                                             C.POINTER(C.c_uint64)]),
    "camelot_stage_corun": (C.c_int32, [C.c_int32, C.POINTER(StageDesc), _P, _P, _P, _P, _P, C.c_int64, _P]),
    "camelot_profile_coruns": (C.c_int32, [C.c_int32, C.POINTER(StageDesc), _P, _P, C.c_int32, C.c_int32,
                                           C.c_int32, _P, C.c_int32, C.c_uint64, C.c_int64,
                                           C.POINTER(CorunRecord)]),
    "camelot_predictor_features": (C.c_int32, [C.POINTER(SoloTables), C.c_int32, _P, _P, _P, _P]),
    "camelot_predictor_fit_norm": (C.c_int32, [_P, C.c_int32, _P, _P]),
    "camelot_predictor_standardize": (C.c_int32, [_P, C.c_int32, _P, _P]),
    "camelot_alloc_peak_learned": (C.c_int32, [C.POINTER(Problem), C.POINTER(SoloTables), _P, _P, _P,
                                               C.POINTER(Alloc), _P]),
    "camelot_predictor_forward": (C.c_int32, [_P, _P, C.c_int32, _P, _P]),
    "camelot_predictor_grad": (C.c_int32, [_P, _P, _P, C.c_int32, _P, C.POINTER(C.c_float), _P]),
    "camelot_predictor_adam": (C.c_int32, [_P, _P, _P, _P, C.c_int32, C.c_float, _P]),
    "camelot_predictor_train": (C.c_int32, [_P, _P, _P, C.POINTER(C.c_int32), _P, _P, C.c_int32,
                                            C.c_int32, C.c_int32, _P, C.c_float, _P, _P]),
    "camelot_dt_fit": (C.c_int32, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "camelot_dt_predict": (C.c_int32, [_P, _P, C.c_int32, _P]),
    "camelot_dt_export": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_int32), _P, _P, _P, _P, _P]),
    "camelot_dt_destroy": (None, [_P]),
    "camelot_pipeline_ipc_info": (C.c_int32, [_P, _P, C.POINTER(C.c_int64)]),
    "camelot_ipc_region_create": (C.c_int32, [C.c_int64, C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "camelot_ipc_region_open": (C.c_int32, [_P, C.POINTER(_P)]),
    "camelot_ipc_region_info": (C.c_int32, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "camelot_ipc_handoff_run": (C.c_int32, [_P, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                            C.POINTER(C.c_double)]),
    "camelot_ipc_region_destroy": (C.c_int32, [_P]),
    "camelot_alloc_peak_dt": (C.c_int32, [C.POINTER(Problem), C.POINTER(SoloTables), _P, C.POINTER(Alloc), _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
EXPORTS = sorted(_SIGS)


def _check(rc: int) -> int:
    if rc < 0:
        raise CamelotError(rc, _lib.camelot_last_error().decode())
    return rc


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


# ------------------------------------------------------------------ device / misc
def camelot_version() -> int:
    return _lib.camelot_version()


def camelot_device_query() -> DeviceInfo:
    d = DeviceInfo()
    _check(_lib.camelot_device_query(C.byref(d)))
    return d


# ------------------------------------------------------------------ allocation
class ProblemArrays:
    """Keeps the numpy arrays a Problem points at alive."""

    def __init__(self, *, cu_total, cu_step, max_instances, max_inst_per_stage, batches, qos_ns,
                 hbm_bytes_budget, hbm_bw_budget, lat_ns, bw_bps, mem_bytes, batch_wait_ns=None, inst_max=None):
        self.batches = np.ascontiguousarray(batches, dtype=np.int32)
        self.lat = _i64(lat_ns)
        self.bw = _i64(bw_bps)
        self.mem = _i64(mem_bytes)
        self.wait = None if batch_wait_ns is None else _i64(batch_wait_ns)
        self.inst_max = None if inst_max is None else np.ascontiguousarray(inst_max, dtype=np.int32)
        self.struct = Problem(
            n_stages=self.lat.shape[0], cu_total=cu_total, cu_step=cu_step, max_instances=max_instances,
            max_inst_per_stage=max_inst_per_stage, n_batches=len(self.batches),
            batches=_ptr(self.batches, C.c_int32), qos_ns=int(qos_ns),
            hbm_bytes_budget=int(hbm_bytes_budget), hbm_bw_budget=int(hbm_bw_budget),
            lat_ns=_ptr(self.lat, C.c_int64), bw_bps=_ptr(self.bw, C.c_int64),
            mem_bytes=_ptr(self.mem, C.c_int64),
            batch_wait_ns=_ptr(self.wait, C.c_int64) if self.wait is not None else None,
            inst_max=_ptr(self.inst_max, C.c_int32) if self.inst_max is not None else None)


OBJ_PEAK, OBJ_MIN = 0, 1


def camelot_alloc_sa(problem: ProblemArrays, objective: int, load_num: int = 0, load_den: int = 1,
                     iters: int = 4000, seed: int = 0):
    """Simulated annealing for Eq. 1 (OBJ_PEAK) or Eq. 3 (OBJ_MIN); None when no
    valid state was visited."""
    a = Alloc()
    rc = _lib.camelot_alloc_sa(C.byref(problem.struct), objective, int(load_num), int(load_den), int(iters),
                               int(seed) & ((1 << 64) - 1), C.byref(a))
    if rc == EINFEASIBLE:
        return None
    _check(rc)
    return a


def camelot_alloc_peak(problem: ProblemArrays):
    """Returns the Alloc, or None when infeasible."""
    a = Alloc()
    rc = _lib.camelot_alloc_peak(C.byref(problem.struct), C.byref(a))
    if rc == EINFEASIBLE:
        return None
    _check(rc)
    return a


def camelot_alloc_min(problem: ProblemArrays, load_num: int, load_den: int = 1):
    a = Alloc()
    rc = _lib.camelot_alloc_min(C.byref(problem.struct), int(load_num), int(load_den), C.byref(a))
    if rc == EINFEASIBLE:
        return None
    _check(rc)
    return a


def camelot_alloc_eval(problem: ProblemArrays, batch_index: int, n, cu):
    """Returns (feasible, Alloc) for the given point."""
    a = Alloc()
    a.batch_index = batch_index
    for i, (nn, cc) in enumerate(zip(n, cu)):
        a.n[i] = nn
        a.cu[i] = cc
    rc = _lib.camelot_alloc_eval(C.byref(problem.struct), C.byref(a))
    if rc == EINFEASIBLE:
        return False, a
    _check(rc)
    return True, a


# ------------------------------------------------------------------ stages
def stage_desc(kind: int, dims=(), weights=(), k: int = 0, n_layers: int | None = None) -> StageDesc:
    d = StageDesc()
    d.kind = kind
    dims = list(dims)
    d.n_layers = n_layers if n_layers is not None else max(len(dims) - 1, 0)
    for i, v in enumerate(dims):
        d.dims[i] = v
    d.k = k
    for i, w in enumerate(weights):
        d.weights[i] = int(w)
    return d


def camelot_stage_row_bytes_in(desc: StageDesc) -> int:
    return _check(_lib.camelot_stage_row_bytes_in(C.byref(desc)))


def camelot_stage_row_bytes_out(desc: StageDesc) -> int:
    return _check(_lib.camelot_stage_row_bytes_out(C.byref(desc)))


def camelot_stage_run(desc: StageDesc, in_ptr: int, out_ptr: int, rows: int, n_cus: int = 0,
                      cu_offset: int = 0, reps: int = 1, device: bool = False) -> float:
    """Runs the stage's one-shot kernel over `reps` batches; returns ns per batch from
    HIP events on its stream (device=True: from the device clock, launch excluded)."""
    ns = C.c_double(0.0)
    dns = C.c_double(0.0)
    _check(_lib.camelot_stage_run(C.byref(desc), in_ptr, out_ptr, rows, n_cus, cu_offset, reps, C.byref(ns),
                                  C.byref(dns)))
    return dns.value if device else ns.value


def camelot_stage_run_noalloc(desc: StageDesc, in_ptr: int, out_ptr: int, rows: int, n_cus: int, reps: int = 1,
                              stream: int = 0) -> None:
    """Enqueues the stage's one-shot kernel on `stream` using only the library's
    static device array (no allocation); returns without waiting."""
    _check(_lib.camelot_stage_run_noalloc(C.byref(desc), in_ptr, out_ptr, rows, n_cus, reps, stream or None))


# ------------------------------------------------------------------ pipelines
def pipeline_config(stages, cu, *, cu_offset=0, max_batch=32, batch_target=1, batch_timeout_ns=0,
                    ring_depth=4, handoff=HANDOFF_DEVICE, ingest=INGEST_HOST, max_rows_per_request=1,
                    ingest_capacity=4096, egress_capacity=65536, idle_timeout_ns=20_000_000_000,
                    hbm_budget_bytes=0, side_bytes=0, n_inst=None, out_ipc=False,
                    ipc_handle=None) -> PipelineConfig:
    c = PipelineConfig()
    c.n_stages = len(stages)
    for i, s in enumerate(stages):
        c.stages[i] = s
        c.cu[i] = cu[i]
        c.n_inst[i] = 1 if n_inst is None else int(n_inst[i])
    c.cu_offset = cu_offset
    c.max_batch = max_batch
    c.batch_target = batch_target
    c.batch_timeout_ns = batch_timeout_ns
    c.ring_depth = ring_depth
    c.handoff = handoff
    c.ingest = ingest
    c.max_rows_per_request = max_rows_per_request
    c.ingest_capacity = ingest_capacity
    c.egress_capacity = egress_capacity
    c.idle_timeout_ns = idle_timeout_ns
    c.hbm_budget_bytes = hbm_budget_bytes
    c.side_bytes = side_bytes
    c.out_ipc = 1 if out_ipc else 0
    if ipc_handle is not None:
        h = bytes(ipc_handle)
        assert len(h) == IPC_HANDLE_BYTES
        C.memmove(c.ipc_handle, h, IPC_HANDLE_BYTES)
    return c


def camelot_pipeline_create(cfg: PipelineConfig) -> int:
    h = C.c_void_p()
    _check(_lib.camelot_pipeline_create(C.byref(cfg), C.byref(h)))
    return h.value


def camelot_pipeline_ipc_info(p: int) -> tuple:
    """(exported handle as bytes, setup ns of the export and/or open)."""
    h = (C.c_uint8 * IPC_HANDLE_BYTES)()
    ns = C.c_int64(0)
    _check(_lib.camelot_pipeline_ipc_info(p, C.addressof(h), C.byref(ns)))
    return bytes(h), ns.value


# ------------------------------------------------------------------ cross-process handoff
def camelot_ipc_region_create(slot_bytes: int, depth: int, channels: int) -> tuple:
    """(region handle, exported IPC handle bytes)."""
    h = (C.c_uint8 * IPC_HANDLE_BYTES)()
    r = C.c_void_p()
    _check(_lib.camelot_ipc_region_create(slot_bytes, depth, channels, C.addressof(h), C.byref(r)))
    return r.value, bytes(h)


def camelot_ipc_region_open(handle: bytes) -> int:
    h = (C.c_uint8 * IPC_HANDLE_BYTES).from_buffer_copy(bytes(handle))
    r = C.c_void_p()
    _check(_lib.camelot_ipc_region_open(C.addressof(h), C.byref(r)))
    return r.value


def camelot_ipc_region_info(r: int) -> dict:
    ns = C.c_int64(0)
    ch = C.c_int32(0)
    _check(_lib.camelot_ipc_region_info(r, C.byref(ns), C.byref(ch)))
    return {"setup_ns": ns.value, "channels": ch.value}


def camelot_ipc_handoff_run(r: int, role: int, n_slots: int, cu_offset: int, timeout_ms: int = 10000) -> dict:
    out = (C.c_double * 5)()
    _check(_lib.camelot_ipc_handoff_run(r, role, n_slots, cu_offset, timeout_ms, out))
    raw = bytes(out)
    return {"seconds": out[0], "bytes": out[1], "sum": int.from_bytes(raw[16:24], "little"),
            "xor": int.from_bytes(raw[24:32], "little"), "gbs": out[4]}


def camelot_ipc_region_destroy(r: int) -> None:
    _check(_lib.camelot_ipc_region_destroy(r))


def camelot_pipeline_footprint(p: int) -> int:
    return _lib.camelot_pipeline_footprint(p)


def camelot_pipeline_epoch_ns(p: int) -> int:
    e = C.c_int64()
    _check(_lib.camelot_pipeline_epoch_ns(p, C.byref(e)))
    return e.value


def camelot_pipeline_submit(p: int, query_id: int, payload: np.ndarray, rows: int) -> int:
    """Returns OK or EAGAIN (queue full); raises on other errors."""
    buf = np.ascontiguousarray(payload)
    rc = _lib.camelot_pipeline_submit(p, int(query_id), buf.ctypes.data, int(rows))
    if rc == EAGAIN:
        return EAGAIN
    return _check(rc)


def camelot_pipeline_drain(p: int, max_results: int = 4096, timeout_ns: int = 0):
    """Returns a list of Result structs (possibly empty on timeout)."""
    out = (Result * max_results)()
    n = C.c_int32(0)
    rc = _lib.camelot_pipeline_drain(p, out, max_results, C.byref(n), int(timeout_ns))
    if rc == ETIMEDOUT:
        return []
    _check(rc)
    return out[: n.value]


def camelot_pipeline_drain_latency(p: int, ids: np.ndarray, lat_ns: np.ndarray, timeout_ns: int = 0) -> int:
    """Fills ids (uint64) and lat_ns (int64) arrays from the front; returns the count."""
    n = C.c_int32(0)
    rc = _lib.camelot_pipeline_drain_latency(p, ids.ctypes.data, lat_ns.ctypes.data, min(len(ids), len(lat_ns)),
                                             C.byref(n), int(timeout_ns))
    if rc == ETIMEDOUT:
        return 0
    _check(rc)
    return n.value


def camelot_pipeline_replay(p: int, ids, rows, arrival_ns, payload_row, payload_ptr: int, payload_rows: int):
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
    prow = np.ascontiguousarray(payload_row, dtype=np.int64)
    _check(_lib.camelot_pipeline_replay(p, len(ids), ids.ctypes.data, rows.ctypes.data, arr.ctypes.data,
                                        prow.ctypes.data, payload_ptr, int(payload_rows)))


def camelot_pipeline_submit_replay(p: int, ids, rows, arrival_ns, payload_row, payload: np.ndarray):
    """Starts the library's paced host submitter; keep `payload` (host array) alive
    until every request is submitted (camelot_pipeline_submit_status)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
    prow = np.ascontiguousarray(payload_row, dtype=np.int64)
    assert payload.flags["C_CONTIGUOUS"]
    _check(_lib.camelot_pipeline_submit_replay(p, len(ids), ids.ctypes.data, rows.ctypes.data, arr.ctypes.data,
                                               prow.ctypes.data, payload.ctypes.data, int(payload.shape[0])))


def camelot_pipeline_submit_status(p: int) -> int:
    n = C.c_int64(0)
    _check(_lib.camelot_pipeline_submit_status(p, C.byref(n)))
    return n.value


def camelot_pipeline_stats_get(p: int) -> PipelineStats:
    s = PipelineStats()
    _check(_lib.camelot_pipeline_stats_get(p, C.byref(s)))
    return s


def camelot_pipeline_destroy(p: int) -> int:
    """Returns the number of undelivered rows."""
    u = C.c_uint64(0)
    _check(_lib.camelot_pipeline_destroy(p, C.byref(u)))
    return u.value


# ------------------------------------------------------------------ share bandwidth
STREAM_READ, STREAM_WRITE, STREAM_COPY, STREAM_SPLIT = 0, 1, 2, 3


def camelot_stream_bench(mode: int, nbytes: int, n_cus: int, cu_offset: int = 0, reps: int = 1) -> dict:
    out = (C.c_double * 3)()
    _check(_lib.camelot_stream_bench(mode, nbytes, n_cus, cu_offset, reps, out))
    return {"seconds": out[0], "bytes": out[1], "gbs": out[2]}


# ------------------------------------------------------------------ handoff
def camelot_handoff_bench(mode: int, slot_bytes: int, depth: int, n_slots: int, cu_producer: int = 128,
                          cu_consumer: int = 128) -> dict:
    out = (C.c_double * 5)()
    _check(_lib.camelot_handoff_bench(mode, slot_bytes, depth, n_slots, cu_producer, cu_consumer, out))
    raw = bytes(out)
    s = int.from_bytes(raw[16:24], "little")
    x = int.from_bytes(raw[24:32], "little")
    return {"seconds": out[0], "bytes": out[1], "sum": s, "xor": x, "gbs": out[4]}


def camelot_handoff_expected(slot_bytes: int, n_slots: int):
    s, x = C.c_uint64(0), C.c_uint64(0)
    _check(_lib.camelot_handoff_expected(slot_bytes, n_slots, C.byref(s), C.byref(x)))
    return s.value, x.value


# ------------------------------------------------------------------ predictor
def camelot_predictor_forward(params: int, x: int, m: int, yhat: int, stream: int = 0):
    _check(_lib.camelot_predictor_forward(params, x, m, yhat, stream or None))


def camelot_predictor_grad(params: int, x: int, y: int, m: int, grad: int, stream: int = 0) -> float:
    loss = C.c_float(0.0)
    _check(_lib.camelot_predictor_grad(params, x, y, m, grad, C.byref(loss), stream or None))
    return loss.value


def camelot_predictor_adam(params: int, grad: int, m1: int, m2: int, t: int, lr: float, stream: int = 0):
    _check(_lib.camelot_predictor_adam(params, grad, m1, m2, t, lr, stream or None))


def camelot_predictor_train(params: int, m1: int, m2: int, t: int, x: int, y: int, n: int, batch: int,
                            epochs: int, perm: int = 0, lr: float = 1e-3, stream: int = 0):
    """Returns (new step counter, per-epoch mean loss array)."""
    tt = C.c_int32(t)
    losses = np.zeros(max(epochs, 1), np.float32)
    _check(_lib.camelot_predictor_train(params, m1, m2, C.byref(tt), x, y, n, batch, epochs, perm or None,
                                        lr, losses.ctypes.data, stream or None))
    return tt.value, losses[:epochs]


# ------------------------------------------------------------------ contention profiles
def _descs(stages):
    arr = (StageDesc * len(stages))()
    for i, s in enumerate(stages):
        arr[i] = s
    return arr


def _ptrs(vals):
    return np.ascontiguousarray([int(v) for v in vals], dtype=np.uint64)


def camelot_stage_corun(stages, ins, outs, rows, n_cus, cu_offset, duration_ns: int):
    """Runs the stages at once on disjoint shares; returns ns per batch of each."""
    n = len(stages)
    d = _descs(stages)
    pin, pout = _ptrs(ins), _ptrs(outs)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(n_cus, dtype=np.int32)
    o = np.ascontiguousarray(cu_offset, dtype=np.int32)
    ns = np.zeros(n, np.float64)
    _check(_lib.camelot_stage_corun(n, d, pin.ctypes.data, pout.ctypes.data, r.ctypes.data, c.ctypes.data,
                                    o.ctypes.data, int(duration_ns), ns.ctypes.data))
    return ns


def camelot_profile_coruns(stages, ins, outs, cu_total, cu_step, batches, n_runs, seed, duration_ns):
    """Random co-location profiles; returns a list of CorunRecord."""
    d = _descs(stages)
    pin, pout = _ptrs(ins), _ptrs(outs)
    b = np.ascontiguousarray(batches, dtype=np.int32)
    recs = (CorunRecord * max(n_runs, 1))()
    _check(_lib.camelot_profile_coruns(len(stages), d, pin.ctypes.data, pout.ctypes.data, cu_total, cu_step,
                                       len(b), b.ctypes.data, n_runs, seed, int(duration_ns), recs))
    return list(recs[:n_runs])


class SoloTablesArrays:
    """Keeps the arrays a SoloTables points at alive. hbm/mfma: [kinds][shares][batches]."""

    def __init__(self, cu_step, batches, hbm, mfma):
        self.batches = np.ascontiguousarray(batches, dtype=np.int32)
        self.hbm = np.ascontiguousarray(hbm, dtype=np.float32)
        self.mfma = np.ascontiguousarray(mfma, dtype=np.float32)
        k, s, b = self.hbm.shape
        self.struct = SoloTables(n_kinds=k, cu_step=cu_step, n_shares=s, n_batches=b,
                                 batches=_ptr(self.batches, C.c_int32),
                                 hbm=_ptr(self.hbm, C.c_float), mfma=_ptr(self.mfma, C.c_float))


def camelot_predictor_features(tables: SoloTablesArrays, kinds, cu, bi) -> np.ndarray:
    m = len(kinds)
    k = np.ascontiguousarray(kinds, dtype=np.int32)
    c = np.ascontiguousarray(cu, dtype=np.int32)
    b = np.ascontiguousarray(bi, dtype=np.int32)
    out = np.zeros((m, 16), np.float32)
    _check(_lib.camelot_predictor_features(C.byref(tables.struct), m, k.ctypes.data, c.ctypes.data,
                                           b.ctypes.data, out.ctypes.data))
    return out


def camelot_predictor_fit_norm(x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.float32)
    mean = np.zeros(16, np.float32)
    std = np.zeros(16, np.float32)
    _check(_lib.camelot_predictor_fit_norm(x.ctypes.data, x.shape[0], mean.ctypes.data, std.ctypes.data))
    return mean, std


def camelot_predictor_standardize(x: np.ndarray, mean, std) -> np.ndarray:
    """Returns a standardised copy."""
    x = np.array(x, dtype=np.float32, order="C", copy=True)
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    std = np.ascontiguousarray(std, dtype=np.float32)
    _check(_lib.camelot_predictor_standardize(x.ctypes.data, x.shape[0], mean.ctypes.data, std.ctypes.data))
    return x


class DecisionTree:
    """A fitted camelot_dt (include/camelot.h); freed with the object."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.camelot_dt_destroy(self._h)
            self._h = None

    def predict(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty(x.shape[0], np.float32)
        _check(_lib.camelot_dt_predict(self._h, x.ctypes.data, x.shape[0], out.ctypes.data))
        return out

    def export(self) -> dict:
        """Nodes in creation order: feat (-1 leaf), thr, value, left, right."""
        n = C.c_int32(0)
        _check(_lib.camelot_dt_export(self._h, 0, C.byref(n), None, None, None, None, None))
        m = n.value
        feat, left, right = (np.empty(m, np.int32) for _ in range(3))
        thr, value = np.empty(m, np.float64), np.empty(m, np.float64)
        _check(_lib.camelot_dt_export(self._h, m, C.byref(n), feat.ctypes.data, thr.ctypes.data,
                                      value.ctypes.data, left.ctypes.data, right.ctypes.data))
        return {"feat": feat, "thr": thr, "value": value, "left": left, "right": right}


def camelot_dt_fit(x, y, max_depth: int, min_leaf: int) -> DecisionTree:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    h = _P()
    _check(_lib.camelot_dt_fit(x.ctypes.data, y.ctypes.data, x.shape[0], x.shape[1], max_depth, min_leaf,
                               C.byref(h)))
    return DecisionTree(h)


def camelot_alloc_peak_learned(problem: ProblemArrays, tables: SoloTablesArrays, params_ptr: int, mean, std):
    """Returns (Alloc or None, predicted stage latencies in ns)."""
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    std = np.ascontiguousarray(std, dtype=np.float32)
    a = Alloc()
    lat = np.zeros(MAX_STAGES, np.int64)
    rc = _lib.camelot_alloc_peak_learned(C.byref(problem.struct), C.byref(tables.struct), params_ptr,
                                         mean.ctypes.data, std.ctypes.data, C.byref(a), lat.ctypes.data)
    if rc == EINFEASIBLE:
        return None, None
    _check(rc)
    return a, lat[: problem.struct.n_stages]


def camelot_alloc_peak_dt(problem: ProblemArrays, tables: SoloTablesArrays, tree: DecisionTree):
    """Returns (Alloc or None, predicted stage latencies in ns)."""
    a = Alloc()
    lat = np.zeros(MAX_STAGES, np.int64)
    rc = _lib.camelot_alloc_peak_dt(C.byref(problem.struct), C.byref(tables.struct), tree._h, C.byref(a),
                                    lat.ctypes.data)
    if rc == EINFEASIBLE:
        return None, None
    _check(rc)
    return a, lat[: problem.struct.n_stages]


# ------------------------------------------------------------------ serving
def camelot_server_create(hbm_budget_bytes: int) -> int:
    h = C.c_void_p()
    _check(_lib.camelot_server_create(int(hbm_budget_bytes), C.byref(h)))
    return h.value


def camelot_server_admit(server: int, cfg: PipelineConfig):
    """Returns the pipeline handle, or None when it does not fit the HBM budget."""
    h = C.c_void_p()
    rc = _lib.camelot_server_admit(server, C.byref(cfg), C.byref(h))
    if rc == ENOMEM:
        return None
    _check(rc)
    return h.value


def camelot_server_release(server: int, p: int) -> int:
    u = C.c_uint64(0)
    _check(_lib.camelot_server_release(server, p, C.byref(u)))
    return u.value


def camelot_server_used_bytes(server: int) -> int:
    return _lib.camelot_server_used_bytes(server)


def camelot_server_destroy(server: int):
    _check(_lib.camelot_server_destroy(server))


def camelot_stage_weight_bytes(desc: StageDesc) -> int:
    return _check(_lib.camelot_stage_weight_bytes(C.byref(desc)))


def camelot_stage_kernel_info(kind: int, one_shot: bool) -> dict:
    regs, lds, fits = C.c_int32(0), C.c_int64(0), C.c_int32(0)
    _check(_lib.camelot_stage_kernel_info(kind, int(one_shot), C.byref(regs), C.byref(lds), C.byref(fits)))
    return {"regs": regs.value, "lds_bytes": lds.value, "fits": bool(fits.value)}
