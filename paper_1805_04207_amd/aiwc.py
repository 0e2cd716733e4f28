"""ctypes binding of libaiwc (include/aiwc.h): argument marshalling only.

Every metric is computed by the HIP kernels inside libaiwc.so; this module
only converts Python / torch objects to the C structs and back.  Importing
it raises if the library is not built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaiwc.so")

AIWC_OK, AIWC_ERR_INVALID_ARG, AIWC_ERR_INCONSISTENT = 0, 1, 2
AIWC_ERR_OUT_OF_MEMORY, AIWC_ERR_HIP, AIWC_ERR_UNSUPPORTED = 3, 4, 5
AIWC_VALIDATE_ON_DEVICE = 1
BRANCH_ZERO_HISTORY, BRANCH_GLOBAL_HISTORY, BRANCH_PATTERN_ENTROPY = 2, 4, 8
STREAM_HOST_RETAIN = 1
SIZING_BOUND, SIZING_HEURISTIC, SIZING_LEARNED = 0, 1, 2
AUTOTUNE_OFF, AUTOTUNE_CACHED, AUTOTUNE_SEARCH = 0, 1, 2
N_FEATURES, N_TARGETS = 40, 11


class AiwcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"aiwc status {status}: {msg}")
        self.status = status


class OpcodeInfo(ctypes.Structure):
    _fields_ = [("op_class", ctypes.c_uint16), ("simd_width", ctypes.c_uint8),
                ("kind", ctypes.c_uint8)]


class TraceDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("n_events", ctypes.c_uint64), ("opcode", ctypes.c_void_p),
                ("n_workitems", ctypes.c_uint64), ("wi_offsets", ctypes.c_void_p),
                ("wg_size", ctypes.c_uint32), ("n_opcode_ids", ctypes.c_uint32),
                ("opcode_table", ctypes.c_void_p), ("n_mem", ctypes.c_uint64),
                ("addr", ctypes.c_void_p), ("mem_kind", ctypes.c_void_p),
                ("n_branch", ctypes.c_uint64), ("br_site", ctypes.c_void_p),
                ("br_taken", ctypes.c_void_p), ("n_sites", ctypes.c_uint32),
                ("history_len", ctypes.c_uint32), ("max_lsb_skip", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class SpaceMetrics(ctypes.Structure):
    _fields_ = [("total_accesses", ctypes.c_uint64), ("total_reads", ctypes.c_uint64),
                ("total_writes", ctypes.c_uint64), ("unique_reads", ctypes.c_uint64),
                ("unique_writes", ctypes.c_uint64), ("footprint", ctypes.c_uint64),
                ("footprint_90", ctypes.c_uint64), ("distinct", ctypes.c_uint64 * 11),
                ("entropy", ctypes.c_double * 11), ("unique_rw_ratio", ctypes.c_double),
                ("reread_ratio", ctypes.c_double), ("rewrite_ratio", ctypes.c_double)]


class MetricsHost(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("history_len", ctypes.c_uint32),
                ("total_instructions", ctypes.c_uint64), ("unique_opcodes", ctypes.c_uint32),
                ("opcodes_90", ctypes.c_uint32), ("simd_max", ctypes.c_uint64),
                ("simd_sum", ctypes.c_uint64), ("simd_sumsq_lo", ctypes.c_uint64),
                ("simd_sumsq_hi", ctypes.c_uint64), ("simd_mean", ctypes.c_double),
                ("simd_sd", ctypes.c_double), ("work_items", ctypes.c_uint64),
                ("barriers_hit", ctypes.c_uint64), ("itb_count", ctypes.c_uint64),
                ("itb_sum", ctypes.c_uint64), ("itb_min", ctypes.c_uint64),
                ("itb_max", ctypes.c_uint64), ("itb_median", ctypes.c_double),
                ("ipt_min", ctypes.c_uint64), ("ipt_max", ctypes.c_uint64),
                ("ipt_median", ctypes.c_double), ("space", SpaceMetrics * 2),
                ("total_branches", ctypes.c_uint64), ("unique_branches", ctypes.c_uint64),
                ("branches_90", ctypes.c_uint64), ("n_windows", ctypes.c_uint64),
                ("albe_min_sum", ctypes.c_uint64), ("yokota_entropy", ctypes.c_double),
                ("linear_branch_entropy", ctypes.c_double),
                ("pattern_entropy", ctypes.c_double), ("granularity", ctypes.c_double),
                ("barriers_per_instruction", ctypes.c_double),
                ("instructions_per_operand", ctypes.c_double),
                ("load_imbalance", ctypes.c_uint64), ("overflow_redos", ctypes.c_uint32),
                ("partitions", ctypes.c_uint32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("sizing", ctypes.c_uint32),
                ("autotune", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("admission_cap_bytes", ctypes.c_uint64),
                ("force_partition_log2", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("waves", ctypes.c_uint32),
                ("reserved_bytes", ctypes.c_uint64), ("redo_partitions", ctypes.c_uint64),
                ("total_partitions", ctypes.c_uint64), ("plan_ms", ctypes.c_double)]


class StreamStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("groups", ctypes.c_uint32),
                ("memory_events", ctypes.c_uint64), ("device_records", ctypes.c_uint64),
                ("largest_partition", ctypes.c_uint64)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("epochs", ctypes.c_uint32),
                ("batch", ctypes.c_uint32), ("seed", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("reserved", ctypes.c_uint32)]


class ProgramDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_insn", ctypes.c_uint32),
                ("code", ctypes.c_void_p), ("n_opcode_ids", ctypes.c_uint32),
                ("n_sites", ctypes.c_uint32), ("opcode_table", ctypes.c_void_p)]


class KernelArg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("ptr", ctypes.c_void_p),
                ("bytes", ctypes.c_uint64), ("value", ctypes.c_uint64)]


class NDRange(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_uint32), ("global_size", ctypes.c_uint32 * 3),
                ("local_size", ctypes.c_uint32 * 3), ("reserved", ctypes.c_uint32)]


ARG_GLOBAL, ARG_LOCAL, ARG_SCALAR = 0, 1, 2


EXPORTS = [
    "aiwc_context_create", "aiwc_context_destroy", "aiwc_last_error", "aiwc_trace_create",
    "aiwc_trace_destroy", "aiwc_characterize", "aiwc_characterize_static",
    "aiwc_characterize_merged",
    "aiwc_stream_create", "aiwc_stream_append", "aiwc_stream_finish", "aiwc_stream_destroy",
    "aiwc_stream_set_device_budget", "aiwc_stream_get_stats",
    "aiwc_characterize_batch", "aiwc_batch_last_stats",
    "aiwc_metrics_read", "aiwc_metrics_class_hist", "aiwc_metrics_spectrum", "aiwc_metrics_destroy",
    "aiwc_sizer_features", "aiwc_sizer_train", "aiwc_sizer_predict", "aiwc_sizer_grad",
    "aiwc_sizer_num_params", "aiwc_sizer_get_params", "aiwc_sizer_set_params", "aiwc_sizer_save",
    "aiwc_sizer_load", "aiwc_sizer_set_margin", "aiwc_profile_enable", "aiwc_profile_read",
    "aiwc_program_create", "aiwc_program_destroy", "aiwc_produce", "aiwc_produced_desc",
    "aiwc_produced_to_host", "aiwc_produced_destroy",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libaiwc.so and declare every export.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library binds to it and one runtime serves the whole process
    # (loading ours first would leave torch with a runtime it cannot use)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, u64, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "aiwc_context_create": (st, [ctypes.c_int, ctypes.POINTER(vp)]),
        "aiwc_context_destroy": (st, [vp]),
        "aiwc_last_error": (ctypes.c_char_p, [vp]),
        "aiwc_trace_create": (st, [vp, ctypes.POINTER(TraceDesc), ctypes.POINTER(vp)]),
        "aiwc_trace_destroy": (st, [vp]),
        "aiwc_characterize": (st, [vp, vp, vp, ctypes.POINTER(vp)]),
        "aiwc_characterize_static": (st, [vp, vp, vp, vp, sz]),
        "aiwc_characterize_merged": (st, [vp, ctypes.POINTER(vp), sz, vp, ctypes.POINTER(vp)]),
        "aiwc_stream_create": (st, [vp, u64, u64, ctypes.c_uint32, ctypes.POINTER(vp)]),
        "aiwc_stream_append": (st, [vp, vp, vp]),
        "aiwc_stream_finish": (st, [vp, vp, ctypes.POINTER(vp)]),
        "aiwc_stream_destroy": (st, [vp]),
        "aiwc_stream_set_device_budget": (st, [vp, u64]),
        "aiwc_stream_get_stats": (st, [vp, ctypes.POINTER(StreamStats)]),
        "aiwc_characterize_batch": (st, [vp, ctypes.POINTER(vp), sz, ctypes.POINTER(BatchOpts), vp,
                                         ctypes.POINTER(vp)]),
        "aiwc_batch_last_stats": (st, [vp, ctypes.POINTER(BatchStats)]),
        "aiwc_metrics_read": (st, [vp, ctypes.POINTER(MetricsHost)]),
        "aiwc_metrics_class_hist": (st, [vp, vp, sz]),
        "aiwc_metrics_spectrum": (st, [vp, ctypes.c_int, vp, vp, sz, ctypes.POINTER(sz)]),
        "aiwc_metrics_destroy": (st, [vp]),
        "aiwc_sizer_features": (st, [vp, ctypes.POINTER(vp), sz, vp, vp]),
        "aiwc_sizer_train": (st, [vp, vp, vp, sz, ctypes.POINTER(TrainOpts), vp,
                                  ctypes.POINTER(ctypes.c_float)]),
        "aiwc_sizer_predict": (st, [vp, vp, sz, vp, vp]),
        "aiwc_sizer_grad": (st, [vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float), vp]),
        "aiwc_sizer_num_params": (sz, []),
        "aiwc_sizer_get_params": (st, [vp, vp]),
        "aiwc_sizer_set_params": (st, [vp, vp]),
        "aiwc_sizer_save": (st, [vp, ctypes.c_char_p]),
        "aiwc_sizer_load": (st, [vp, ctypes.c_char_p]),
        "aiwc_sizer_set_margin": (st, [vp, ctypes.c_float]),
        "aiwc_profile_enable": (st, [vp, ctypes.c_int]),
        "aiwc_profile_read": (st, [vp, ctypes.c_char_p, sz, vp, sz, ctypes.POINTER(sz)]),
        "aiwc_program_create": (st, [vp, ctypes.POINTER(ProgramDesc), ctypes.POINTER(vp)]),
        "aiwc_program_destroy": (st, [vp]),
        "aiwc_produce": (st, [vp, ctypes.POINTER(NDRange), vp, ctypes.c_uint32, u64, vp,
                              ctypes.POINTER(vp)]),
        "aiwc_produced_desc": (st, [vp, ctypes.POINTER(TraceDesc)]),
        "aiwc_produced_to_host": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "aiwc_produced_destroy": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _struct_to_dict(s) -> Dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        if isinstance(v, ctypes.Array):
            if len(v) and isinstance(v[0], ctypes.Structure):
                out[name] = [_struct_to_dict(x) for x in v]
            else:
                out[name] = list(v)
        else:
            out[name] = v
    return out


class Context:
    """aiwc_ctx: owns scratch, the tuning cache and the sizing network."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.aiwc_context_create(device, ctypes.byref(h))
        if st != AIWC_OK:
            raise AiwcError(st, self.lib.aiwc_last_error(None).decode())
        self.h = h
        self.device = device

    def check(self, st: int):
        if st != AIWC_OK:
            raise AiwcError(st, self.lib.aiwc_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.lib.aiwc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- traces
    def trace(self, opcode, wi_offsets, addr, mem_kind, br_site, br_taken, table,
              n_sites: int, history_len: int = 16, wg_size: int = 0,
              validate: bool = False, branch_flags: int = 0) -> "Trace":
        """Describe a trace held in torch CUDA tensors (device memory).
        branch_flags: BRANCH_* variant bits."""
        return Trace(self, opcode, wi_offsets, addr, mem_kind, br_site, br_taken, table,
                     n_sites, history_len, wg_size, validate, branch_flags)

    def characterize(self, trace: "Trace", stream=None) -> "Metrics":
        m = ctypes.c_void_p()
        self.check(self.lib.aiwc_characterize(self.h, trace.h, _stream_ptr(stream),
                                              ctypes.byref(m)))
        return Metrics(self, m)

    def characterize_static(self, trace: "Trace", out, stream=None):
        """aiwc_characterize_static: no allocation; the result goes to `out`,
        a uint8 CUDA tensor of at least static_result_bytes(n_classes) bytes
        (decode a host copy with static_result)."""
        self.check(self.lib.aiwc_characterize_static(self.h, trace.h, _stream_ptr(stream),
                                                     out.data_ptr(), int(out.numel())))

    def characterize_merged(self, traces: Sequence["Trace"], stream=None) -> "Metrics":
        """Metrics of the invocations taken together (their concatenation)."""
        n = len(traces)
        arr = (ctypes.c_void_p * max(1, n))(*[t.h.value for t in traces])
        m = ctypes.c_void_p()
        self.check(self.lib.aiwc_characterize_merged(self.h, arr, n, _stream_ptr(stream),
                                                     ctypes.byref(m)))
        return Metrics(self, m)

    def program(self, code, table, n_sites: int) -> "Program":
        """A kernel program for the trace producer (aiwc_program_create)."""
        return Program(self, code, table, n_sites)

    def stream(self, mem_hint: int = 0, branch_hint: int = 0,
               host_retain: bool = False) -> "Stream":
        """A trace that arrives in chunks (aiwc_stream_*); the hints reserve
        the retained buffers for that many memory / branch events; with
        host_retain they are kept in pinned host memory until finish."""
        return Stream(self, mem_hint, branch_hint, STREAM_HOST_RETAIN if host_retain else 0)

    def characterize_batch(self, traces: Sequence["Trace"], sizing: int = SIZING_BOUND,
                           autotune: int = AUTOTUNE_OFF, use_graph: bool = False,
                           admission_cap_bytes: int = 0, force_partition_log2: int = 0,
                           stream=None) -> List["Metrics"]:
        n = len(traces)
        arr = (ctypes.c_void_p * max(1, n))(*[t.h.value for t in traces])
        outs = (ctypes.c_void_p * max(1, n))()
        o = BatchOpts(ctypes.sizeof(BatchOpts), sizing, autotune, int(use_graph),
                      admission_cap_bytes, force_partition_log2, 0)
        self.check(self.lib.aiwc_characterize_batch(self.h, arr, n, ctypes.byref(o),
                                                    _stream_ptr(stream), outs))
        return [Metrics(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def batch_stats(self) -> Dict:
        s = BatchStats()
        s.struct_size = ctypes.sizeof(BatchStats)
        self.check(self.lib.aiwc_batch_last_stats(self.h, ctypes.byref(s)))
        return _struct_to_dict(s)

    # --------------------------------------------------------- instrumentation
    def profile_enable(self, on: bool = True):
        self.check(self.lib.aiwc_profile_enable(self.h, int(on)))

    def profile_read(self):
        """[(kernel name, ms)] of the context's last characterization."""
        import numpy as np
        names = ctypes.create_string_buffer(4096)
        ms = np.zeros(64, dtype=np.float64)
        n = ctypes.c_size_t()
        self.check(self.lib.aiwc_profile_read(self.h, names, 4096, ms.ctypes.data, 64,
                                              ctypes.byref(n)))
        lab = names.value.decode().split(",") if n.value else []
        return list(zip(lab, ms[:n.value].tolist()))

    # ---------------------------------------------------------------- sizer
    def sizer_features(self, traces: Sequence["Trace"], out, stream=None):
        n = len(traces)
        arr = (ctypes.c_void_p * max(1, n))(*[t.h.value for t in traces])
        self.check(self.lib.aiwc_sizer_features(self.h, arr, n, _stream_ptr(stream),
                                                out.data_ptr()))

    def sizer_train(self, x, y, epochs: int = 50, batch: int = 256, lr: float = 1e-3,
                    seed: int = 0, stream=None) -> float:
        o = TrainOpts(ctypes.sizeof(TrainOpts), epochs, batch, seed, lr, 0.9, 0.999, 1e-8, 0)
        loss = ctypes.c_float()
        self.check(self.lib.aiwc_sizer_train(self.h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                             ctypes.byref(o), _stream_ptr(stream),
                                             ctypes.byref(loss)))
        return loss.value

    def sizer_predict(self, x, out, stream=None):
        self.check(self.lib.aiwc_sizer_predict(self.h, x.data_ptr(), x.shape[0],
                                               _stream_ptr(stream), out.data_ptr()))

    def sizer_grad(self, xn, yn, stream=None):
        import numpy as np
        n = self.lib.aiwc_sizer_num_params()
        g = np.zeros(n, dtype=np.float32)
        loss = ctypes.c_float()
        self.check(self.lib.aiwc_sizer_grad(self.h, xn.data_ptr(), yn.data_ptr(), xn.shape[0],
                                            _stream_ptr(stream), ctypes.byref(loss),
                                            g.ctypes.data))
        return loss.value, g

    def sizer_params(self):
        import numpy as np
        p = np.zeros(self.lib.aiwc_sizer_num_params(), dtype=np.float32)
        self.check(self.lib.aiwc_sizer_get_params(self.h, p.ctypes.data))
        return p

    def sizer_set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        self.check(self.lib.aiwc_sizer_set_params(self.h, p.ctypes.data))

    def sizer_save(self, path: str):
        self.check(self.lib.aiwc_sizer_save(self.h, path.encode()))

    def sizer_load(self, path: str):
        self.check(self.lib.aiwc_sizer_load(self.h, path.encode()))

    def sizer_set_margin(self, margin_log2: float):
        self.check(self.lib.aiwc_sizer_set_margin(self.h, margin_log2))


STATIC_SCRATCH_BYTES = 64 << 20


def static_class_offset() -> int:
    """AIWC_STATIC_CLASS_OFFSET of include/aiwc.h."""
    return (ctypes.sizeof(MetricsHost) + 32 + 255) // 256 * 256


def static_result_bytes(n_classes: int) -> int:
    """AIWC_STATIC_RESULT_BYTES(n_classes) of include/aiwc.h."""
    return static_class_offset() + 8 * n_classes


def static_result(raw: bytes, n_classes: int):
    """Decode a host copy of an aiwc_characterize_static result block:
    (metrics dict, class histogram list).  The status words map to the
    errors aiwc_metrics_read reports."""
    import numpy as np
    n = ctypes.sizeof(MetricsHost)
    r = MetricsHost.from_buffer_copy(raw[:n])
    status = np.frombuffer(raw[n:n + 32], dtype=np.uint64)
    if status[0]:
        raise AiwcError(AIWC_ERR_INVALID_ARG, f"trace content is invalid ({int(status[0])})")
    if status[1]:
        raise AiwcError(AIWC_ERR_INCONSISTENT, "opcode kinds disagree with the stream lengths")
    if status[3]:
        raise AiwcError(AIWC_ERR_UNSUPPORTED, "an on-chip table round could not be split")
    o = static_class_offset()
    cls = np.frombuffer(raw[o:o + 8 * n_classes], dtype=np.uint64)
    return _struct_to_dict(r), cls.tolist()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Stream:
    """aiwc_stream: append chunk traces, then finish into one Metrics.  The
    chunks' tensors are kept referenced until the stream is closed, since
    the appends read them asynchronously."""

    def __init__(self, ctx: "Context", mem_hint: int = 0, branch_hint: int = 0, flags: int = 0):
        self.ctx = ctx
        self.h = ctypes.c_void_p()
        self._keep = []
        ctx.check(ctx.lib.aiwc_stream_create(ctx.h, mem_hint, branch_hint, flags,
                                             ctypes.byref(self.h)))

    def append(self, chunk: "Trace", stream=None):
        self._keep.append(chunk)
        self.ctx.check(self.ctx.lib.aiwc_stream_append(self.h, chunk.h, _stream_ptr(stream)))

    def set_device_budget(self, nbytes: int):
        """Cap the device bytes finish may use for partition records (0: no
        cap); above it the memory stage runs group by group."""
        self.ctx.check(self.ctx.lib.aiwc_stream_set_device_budget(self.h, int(nbytes)))

    def stats(self) -> Dict:
        s = StreamStats()
        s.struct_size = ctypes.sizeof(StreamStats)
        self.ctx.check(self.ctx.lib.aiwc_stream_get_stats(self.h, ctypes.byref(s)))
        return _struct_to_dict(s)

    def finish(self, stream=None) -> "Metrics":
        m = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.aiwc_stream_finish(self.h, _stream_ptr(stream),
                                                       ctypes.byref(m)))
        return Metrics(self.ctx, m, keep=self)

    def close(self):
        if self.h:
            self.ctx.lib.aiwc_stream_destroy(self.h)
            self.h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trace:
    """aiwc_trace: borrows the tensors (kept referenced here)."""

    def __init__(self, ctx: Context, opcode, wi_offsets, addr, mem_kind, br_site, br_taken,
                 table, n_sites, history_len, wg_size, validate, branch_flags=0):
        import numpy as np
        self.ctx = ctx
        self._keep = (opcode, wi_offsets, addr, mem_kind, br_site, br_taken)
        tab = np.asarray(table)
        self._table = (OpcodeInfo * len(tab))()
        for i, e in enumerate(tab):
            self._table[i] = OpcodeInfo(int(e["op_class"]), int(e["simd_width"]), int(e["kind"]))
        n_wi = int(wi_offsets.numel()) - 1
        d = TraceDesc()
        d.struct_size = ctypes.sizeof(TraceDesc)
        d.flags = (AIWC_VALIDATE_ON_DEVICE if validate else 0) | int(branch_flags)
        d.n_events = _n(opcode)
        d.opcode = _ptr(opcode)
        d.n_workitems = n_wi
        d.wi_offsets = _ptr(wi_offsets)
        d.wg_size = wg_size
        d.n_opcode_ids = len(tab)
        d.opcode_table = ctypes.cast(self._table, ctypes.c_void_p)
        d.n_mem = _n(addr)
        d.addr = _ptr(addr)
        d.mem_kind = _ptr(mem_kind)
        d.n_branch = _n(br_site)
        d.br_site = _ptr(br_site)
        d.br_taken = _ptr(br_taken)
        d.n_sites = n_sites
        d.history_len = history_len
        d.max_lsb_skip = 10
        self.desc = d
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.aiwc_trace_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.ctx.lib.aiwc_trace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _n(t) -> int:
    return 0 if t is None else int(t.numel())


def _ptr(t) -> Optional[int]:
    return None if t is None or t.numel() == 0 else t.data_ptr()


class Metrics:
    """aiwc_metrics: a pending result on the device."""

    def __init__(self, ctx: Context, h, keep=None):
        self.ctx = ctx
        self.h = h
        self._keep = keep   # an object whose buffers the pending work reads

    def read(self) -> Dict:
        r = MetricsHost()
        self.ctx.check(self.ctx.lib.aiwc_metrics_read(self.h, ctypes.byref(r)))
        return _struct_to_dict(r)

    def class_hist(self, n: int):
        import numpy as np
        out = np.zeros(n, dtype=np.uint64)
        self.ctx.check(self.ctx.lib.aiwc_metrics_class_hist(self.h, out.ctypes.data, n))
        return out

    def spectrum(self, space: int):
        import numpy as np
        n = ctypes.c_size_t()
        self.ctx.check(self.ctx.lib.aiwc_metrics_spectrum(self.h, space, None, None, 0,
                                                          ctypes.byref(n)))
        f = np.zeros(max(1, n.value), dtype=np.uint64)
        m = np.zeros(max(1, n.value), dtype=np.uint64)
        self.ctx.check(self.ctx.lib.aiwc_metrics_spectrum(self.h, space, f.ctypes.data,
                                                          m.ctypes.data, n.value,
                                                          ctypes.byref(n)))
        return [(int(a), int(b)) for a, b in zip(f[:n.value], m[:n.value])]

    def close(self):
        if self.h:
            self.ctx.lib.aiwc_metrics_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Program:
    """aiwc_program: a kernel program (24-byte instruction records, numpy)
    with its opcode table and number of branch sites."""

    def __init__(self, ctx: Context, code, table, n_sites: int):
        import numpy as np
        self.ctx = ctx
        self._code = np.ascontiguousarray(code)
        if self._code.dtype.itemsize != 24:
            raise ValueError("instruction records are 24 bytes")
        tab = np.asarray(table)
        self._table = (OpcodeInfo * len(tab))()
        for i, e in enumerate(tab):
            self._table[i] = OpcodeInfo(int(e["op_class"]), int(e["simd_width"]), int(e["kind"]))
        d = ProgramDesc(ctypes.sizeof(ProgramDesc), self._code.size, self._code.ctypes.data,
                        len(tab), int(n_sites), ctypes.cast(self._table, ctypes.c_void_p))
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.aiwc_program_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h

    def produce(self, global_size, local_size, args, max_steps: int = 0, stream=None) -> "Produced":
        """Run the program; args are (ARG_GLOBAL, cuda tensor), (ARG_LOCAL,
        bytes) or (ARG_SCALAR, value) pairs.  Global tensors are updated."""
        n = len(args)
        ca = (KernelArg * max(1, n))()
        for i, (kind, v) in enumerate(args):
            ca[i].kind = kind
            if kind == ARG_GLOBAL:
                ca[i].ptr = v.data_ptr()
                ca[i].bytes = v.numel() * v.element_size()
            elif kind == ARG_LOCAL:
                ca[i].bytes = int(v)
            else:
                ca[i].value = int(v) & 0xFFFFFFFFFFFFFFFF
        nd = NDRange()
        nd.dims = len(global_size)
        for i in range(3):
            nd.global_size[i] = int(global_size[i]) if i < len(global_size) else 1
            nd.local_size[i] = int(local_size[i]) if i < len(local_size) else 1
        h = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.aiwc_produce(self.h, ctypes.byref(nd), ca, n, int(max_steps),
                                                 _stream_ptr(stream), ctypes.byref(h)))
        return Produced(self.ctx, h)

    def close(self):
        if self.h:
            self.ctx.lib.aiwc_program_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Produced:
    """aiwc_produced: the trace arrays of one launch, on the device."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h
        self.desc = TraceDesc()
        ctx.check(ctx.lib.aiwc_produced_desc(h, ctypes.byref(self.desc)))

    def to_host(self) -> Dict:
        import numpy as np
        d = self.desc
        out = {"opcode": np.zeros(d.n_events, np.uint16),
               "wi_offsets": np.zeros(d.n_workitems + 1, np.uint64),
               "addr": np.zeros(d.n_mem, np.uint64), "mem_kind": np.zeros(d.n_mem, np.uint8),
               "br_site": np.zeros(d.n_branch, np.uint32),
               "br_taken": np.zeros(d.n_branch, np.uint8)}
        keys = ("opcode", "wi_offsets", "addr", "mem_kind", "br_site", "br_taken")
        self.ctx.check(self.ctx.lib.aiwc_produced_to_host(self.h, *[out[k].ctypes.data for k in keys]))
        return out

    def trace(self, history_len: int = 16, branch_flags: int = 0) -> "ProducedTrace":
        return ProducedTrace(self, history_len, branch_flags)

    def close(self):
        if self.h:
            self.ctx.lib.aiwc_produced_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ProducedTrace(Trace):
    """aiwc_trace over a produced trace's arrays (keeps the producer alive)."""

    def __init__(self, produced: Produced, history_len: int = 16, branch_flags: int = 0):
        ctx = produced.ctx
        self.ctx = ctx
        self._keep = produced
        d = TraceDesc.from_buffer_copy(produced.desc)
        d.history_len = history_len
        d.flags = int(branch_flags)
        self.desc = d
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.aiwc_trace_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
