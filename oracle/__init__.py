"""CPU oracle for the AIWC metrics -- TEST INFRASTRUCTURE ONLY.

``liboracle.so`` (aiwc_oracle.c) is a plain restatement of the paper's
Table I definitions (arXiv 1805.04207); ``brute.py`` restates them once more
in pure Python with 50-digit mpmath arithmetic for tiny inputs.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build() -> str:
    """Compile the C oracle (gcc, host only)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-ffp-contract=off",
           os.path.join(HERE, "aiwc_oracle.c"), os.path.join(HERE, "producer.c"), "-o", LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


class OrcOpinfo(ctypes.Structure):
    _fields_ = [("op_class", ctypes.c_uint16), ("simd_width", ctypes.c_uint8),
                ("kind", ctypes.c_uint8)]


class OrcTrace(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint64), ("opcode", ctypes.c_void_p),
                ("n_wi", ctypes.c_uint64), ("wi_offsets", ctypes.c_void_p),
                ("n_ids", ctypes.c_uint32), ("n_sites", ctypes.c_uint32),
                ("table", ctypes.c_void_p), ("n_mem", ctypes.c_uint64),
                ("addr", ctypes.c_void_p), ("mem_kind", ctypes.c_void_p),
                ("n_branch", ctypes.c_uint64), ("br_site", ctypes.c_void_p),
                ("br_taken", ctypes.c_void_p), ("history_len", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]

# branch-entropy variants (trace attribute `branch_flags`; the values are the
# interface of the trace flags)
BR_ZERO_HISTORY, BR_GLOBAL_HISTORY, BR_PATTERN = 2, 4, 8


class OrcSpace(ctypes.Structure):
    _fields_ = [("total_accesses", ctypes.c_uint64), ("total_reads", ctypes.c_uint64),
                ("total_writes", ctypes.c_uint64), ("unique_reads", ctypes.c_uint64),
                ("unique_writes", ctypes.c_uint64), ("footprint", ctypes.c_uint64),
                ("footprint_90", ctypes.c_uint64), ("distinct", ctypes.c_uint64 * 11),
                ("entropy", ctypes.c_double * 11), ("unique_rw_ratio", ctypes.c_double),
                ("reread_ratio", ctypes.c_double), ("rewrite_ratio", ctypes.c_double)]


class OrcResult(ctypes.Structure):
    _fields_ = [("total_instructions", ctypes.c_uint64), ("unique_opcodes", ctypes.c_uint64),
                ("opcodes_90", ctypes.c_uint64), ("simd_max", ctypes.c_uint64),
                ("simd_sum", ctypes.c_uint64), ("simd_sumsq_lo", ctypes.c_uint64),
                ("simd_sumsq_hi", ctypes.c_uint64), ("simd_mean", ctypes.c_double),
                ("simd_sd", ctypes.c_double), ("work_items", ctypes.c_uint64),
                ("barriers_hit", ctypes.c_uint64), ("itb_count", ctypes.c_uint64),
                ("itb_sum", ctypes.c_uint64), ("itb_min", ctypes.c_uint64),
                ("itb_max", ctypes.c_uint64), ("itb_median", ctypes.c_double),
                ("ipt_min", ctypes.c_uint64), ("ipt_max", ctypes.c_uint64),
                ("ipt_median", ctypes.c_double), ("space", OrcSpace * 2),
                ("total_branches", ctypes.c_uint64), ("unique_branches", ctypes.c_uint64),
                ("branches_90", ctypes.c_uint64), ("n_windows", ctypes.c_uint64),
                ("albe_min_sum", ctypes.c_uint64), ("yokota_entropy", ctypes.c_double),
                ("linear_branch_entropy", ctypes.c_double),
                ("pattern_entropy", ctypes.c_double), ("granularity", ctypes.c_double),
                ("barriers_per_instruction", ctypes.c_double),
                ("instructions_per_operand", ctypes.c_double),
                ("load_imbalance", ctypes.c_uint64)]


class OrcArg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("host", ctypes.c_void_p),
                ("bytes", ctypes.c_uint64), ("value", ctypes.c_uint64)]


class OrcProduced(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint64), ("n_wi", ctypes.c_uint64),
                ("n_mem", ctypes.c_uint64), ("n_branch", ctypes.c_uint64),
                ("opcode", ctypes.c_void_p), ("wi_offsets", ctypes.c_void_p),
                ("addr", ctypes.c_void_p), ("mem_kind", ctypes.c_void_p),
                ("mem_wi", ctypes.c_void_p), ("br_site", ctypes.c_void_p),
                ("br_taken", ctypes.c_void_p), ("error", ctypes.c_uint32),
                ("error_wi", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_characterize.argtypes = [ctypes.POINTER(OrcTrace), ctypes.POINTER(OrcResult)]
        L.orc_kinds_consistent.argtypes = [ctypes.POINTER(OrcTrace)]
        L.orc_class_hist.argtypes = [ctypes.POINTER(OrcTrace), ctypes.c_void_p, ctypes.c_size_t]
        L.orc_spectrum.argtypes = [ctypes.POINTER(OrcTrace), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_size_t)]
        L.orc_produce.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(OrcProduced)]
        L.orc_produce_free.argtypes = [ctypes.POINTER(OrcProduced)]
        _lib = L
    return _lib


def _as(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


class _Bound:
    """Keeps numpy buffers alive while the C struct points at them."""

    def __init__(self, tr):
        tab = np.asarray(tr.table)
        self.opcode = _as(tr.opcode, np.uint16)
        self.off = _as(tr.wi_offsets, np.uint64)
        self.tab = np.zeros(len(tab), dtype=[("op_class", "<u2"), ("simd_width", "u1"), ("kind", "u1")])
        self.tab["op_class"] = tab["op_class"]
        self.tab["simd_width"] = tab["simd_width"]
        self.tab["kind"] = tab["kind"]
        self.addr = _as(tr.addr, np.uint64)
        self.kind = _as(tr.mem_kind, np.uint8)
        self.site = _as(tr.br_site, np.uint32)
        self.taken = _as(tr.br_taken, np.uint8)
        t = OrcTrace()
        t.n_events = self.opcode.size
        t.opcode = self.opcode.ctypes.data
        t.n_wi = self.off.size - 1
        t.wi_offsets = self.off.ctypes.data
        t.n_ids = len(self.tab)
        t.n_sites = int(tr.n_sites)
        t.table = self.tab.ctypes.data
        t.n_mem = self.addr.size
        t.addr = self.addr.ctypes.data
        t.mem_kind = self.kind.ctypes.data
        t.n_branch = self.site.size
        t.br_site = self.site.ctypes.data
        t.br_taken = self.taken.ctypes.data
        t.history_len = int(tr.history_len)
        t.flags = int(getattr(tr, "branch_flags", 0))
        self.t = t


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


class MergedTrace:
    """Several invocations of one kernel as the one trace they form together.

    The paper reports each kernel as the aggregate over all its invocations
    at a problem size (Evaluation section).  The aggregate is defined here as
    the metrics of the concatenation, in order, of the invocations' work-items
    (instruction streams with their offsets moved behind the events before
    them), memory streams and branch streams; n_sites is the largest of
    theirs.  The opcode table and history length must be the same."""

    def __init__(self, traces):
        traces = list(traces)
        if not traces:
            raise ValueError("no invocations")
        t0 = traces[0]
        tab0 = np.asarray(t0.table)
        for t in traces[1:]:
            if int(t.history_len) != int(t0.history_len) or \
                    int(getattr(t, "branch_flags", 0)) != int(getattr(t0, "branch_flags", 0)) or \
                    not np.array_equal(np.asarray(t.table), tab0):
                raise ValueError("invocations differ in opcode table, history length or "
                                 "branch variant")
        self.table = tab0
        self.history_len = int(t0.history_len)
        self.branch_flags = int(getattr(t0, "branch_flags", 0))
        self.n_sites = max(int(t.n_sites) for t in traces)
        self.opcode = np.concatenate([_as(t.opcode, np.uint16) for t in traces])
        offs, base = [np.zeros(1, dtype=np.uint64)], 0
        for t in traces:
            o = _as(t.wi_offsets, np.uint64)
            offs.append(o[1:] + np.uint64(base))
            base += int(o[-1])
        self.wi_offsets = np.concatenate(offs)
        self.addr = np.concatenate([_as(t.addr, np.uint64) for t in traces])
        self.mem_kind = np.concatenate([_as(t.mem_kind, np.uint8) for t in traces])
        self.br_site = np.concatenate([_as(t.br_site, np.uint32) for t in traces])
        self.br_taken = np.concatenate([_as(t.br_taken, np.uint8) for t in traces])


def characterize_merged(traces) -> Dict:
    """Metrics of several invocations taken together (see MergedTrace)."""
    return characterize(MergedTrace(traces))


def characterize(tr) -> Dict:
    """Metrics of a host trace (any object with the HostTrace attributes)."""
    L = _load()
    b = _Bound(tr)
    r = OrcResult()
    rc = L.orc_characterize(ctypes.byref(b.t), ctypes.byref(r))
    if rc != 0:
        raise ValueError(f"oracle rejected the trace (rc={rc})")
    return _struct_to_dict(r)


def consistent(tr) -> bool:
    """Whether the opcode kinds announce the trace's memory and branch events
    (an atomic read-modify-write is one instruction with two memory events)."""
    L = _load()
    b = _Bound(tr)
    rc = L.orc_kinds_consistent(ctypes.byref(b.t))
    if rc < 0:
        raise ValueError("oracle rejected the trace")
    return rc == 1


def class_hist(tr, n_classes: int) -> np.ndarray:
    L = _load()
    b = _Bound(tr)
    out = np.zeros(n_classes, dtype=np.uint64)
    if L.orc_class_hist(ctypes.byref(b.t), out.ctypes.data, n_classes) != 0:
        raise ValueError("oracle rejected the trace")
    return out


def spectrum(tr, space: int, k: int = 0):
    """Count-of-counts [(f, m_f)] ascending in f."""
    L = _load()
    b = _Bound(tr)
    n = ctypes.c_size_t()
    L.orc_spectrum(ctypes.byref(b.t), space, k, None, None, 0, ctypes.byref(n))
    f = np.zeros(max(1, n.value), dtype=np.uint64)
    m = np.zeros(max(1, n.value), dtype=np.uint64)
    if L.orc_spectrum(ctypes.byref(b.t), space, k, f.ctypes.data, m.ctypes.data, n.value,
                      ctypes.byref(n)) != 0:
        raise ValueError("oracle rejected the trace")
    return [(int(a), int(c)) for a, c in zip(f[:n.value], m[:n.value])]


# ------------------------------------------------------------ trace producer
PRODUCE_ERRORS = {1: "out of bounds", 2: "misaligned", 4: "step limit", 8: "barrier mismatch",
                  16: "ran off the program", 64: "invalid program"}


class ProduceError(RuntimeError):
    def __init__(self, code: int, wi: int):
        super().__init__(f"kernel failed: {PRODUCE_ERRORS.get(code, code)} (work-item {wi})")
        self.code = code
        self.wi = wi


class ProducedTrace:
    """The oracle's trace of one kernel launch (HostTrace attributes, plus
    mem_wi: the work-item of each memory event, in execution order)."""

    def __init__(self, program, arrays, wg_size):
        self.opcode, self.wi_offsets, self.addr, self.mem_kind, self.mem_wi, \
            self.br_site, self.br_taken = arrays
        self.table = program.table
        self.n_sites = max(1, int(program.n_sites))
        self.history_len = 16
        self.wg_size = wg_size


def produce(program, global_size, local_size, args, max_steps: int = 0) -> ProducedTrace:
    """Run `program` (code: 24-byte instruction records, table, n_sites) over
    the ND-range on the CPU in the paper's schedule.  args: Global (numpy
    buffer, updated in place), Local (bytes) or Scalar (64-bit value)
    objects.  Raises ProduceError when the kernel fails."""
    L = _load()
    code = np.ascontiguousarray(program.code)
    assert code.dtype.itemsize == 24
    dims = len(global_size)
    g = (ctypes.c_uint32 * 3)(*(list(global_size) + [1] * (3 - dims)))
    lo = (ctypes.c_uint32 * 3)(*(list(local_size) + [1] * (3 - dims)))
    cargs = (OrcArg * max(1, len(args)))()
    keep = []
    for i, a in enumerate(args):
        kind = a.kind
        cargs[i].kind = kind
        if kind == 0:
            buf = a.array
            assert buf.flags.c_contiguous
            keep.append(buf)
            cargs[i].host = buf.ctypes.data
            cargs[i].bytes = buf.nbytes
        elif kind == 1:
            cargs[i].bytes = int(a.nbytes)
        else:
            cargs[i].value = int(a.value) & 0xFFFFFFFFFFFFFFFF
    out = OrcProduced()
    rc = L.orc_produce(code.ctypes.data, code.size, dims, g, lo, cargs, len(args), max_steps,
                       ctypes.byref(out))
    if rc != 0:
        raise MemoryError("oracle producer ran out of memory")
    if out.error:
        raise ProduceError(out.error, out.error_wi)
    try:
        def arr(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt))),
                                         shape=(n,)).copy()
        arrays = (arr(out.opcode, out.n_events, np.uint16), arr(out.wi_offsets, out.n_wi + 1, np.uint64),
                  arr(out.addr, out.n_mem, np.uint64), arr(out.mem_kind, out.n_mem, np.uint8),
                  arr(out.mem_wi, out.n_mem, np.uint64), arr(out.br_site, out.n_branch, np.uint32),
                  arr(out.br_taken, out.n_branch, np.uint8))
    finally:
        L.orc_produce_free(ctypes.byref(out))
    wg = 1
    for x in local_size:
        wg *= int(x)
    return ProducedTrace(program, arrays, wg)
