"""Seeded synthetic AIWC traces (input generation only).

This module produces the event traces that both the CPU oracle and the HIP
path consume.  It holds none of the characterization arithmetic: the recipe
in ``tg_core.h`` is integer-only (splitmix64 counter hashing + integer
tables built here once), so ``generate_host`` (C, POSIX threads) and
``generate_device`` (HIP) write byte-identical arrays.

The five workloads mirror the paper's workload classes (Demonstration
section: constant-stride, power-of-two-stride, random-gather, barrier-dense
and flag-dominated kernels at L1..DRAM sized footprints) with synthetic
parameters; no benchmark suite data is reproduced.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(HERE, "libtracegen_host.so")
DEV_LIB = os.path.join(HERE, "libtracegen_dev.so")

Q32 = 1 << 32
MASK64 = (1 << 64) - 1

# opcode id layout shared by every generated trace
N_COMPUTE_IDS = 60
ID_LOAD, ID_STORE, ID_BRANCH, ID_BARRIER, ID_RET, ID_ATOMIC = 60, 61, 62, 63, 64, 65
N_OPCODE_IDS = 66
KIND_COMPUTE, KIND_LOAD, KIND_STORE, KIND_ATOMIC, KIND_BRANCH, KIND_BARRIER, KIND_OTHER = range(7)


class TgParams(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("n_wi", ctypes.c_uint64),
        ("wg_size", ctypes.c_uint32), ("len_min", ctypes.c_uint32),
        ("len_max", ctypes.c_uint32), ("barrier_period", ctypes.c_uint32),
        ("p_mem_q32", ctypes.c_uint32), ("p_branch_q32", ctypes.c_uint32),
        ("p_store_q32", ctypes.c_uint32), ("p_local_q32", ctypes.c_uint32),
        ("t_sweep_q32", ctypes.c_uint32), ("t_stencil_q32", ctypes.c_uint32),
        ("sweep_base", ctypes.c_uint64), ("sweep_stride", ctypes.c_uint64),
        ("sweep_words", ctypes.c_uint64), ("stencil_base", ctypes.c_uint64),
        ("stencil_dim", ctypes.c_uint64), ("random_base", ctypes.c_uint64),
        ("random_words", ctypes.c_uint64), ("local_words", ctypes.c_uint64),
        ("n_compute_ids", ctypes.c_uint32), ("id_load", ctypes.c_uint32),
        ("id_store", ctypes.c_uint32), ("id_branch", ctypes.c_uint32),
        ("id_barrier", ctypes.c_uint32), ("id_ret", ctypes.c_uint32),
        ("n_sites", ctypes.c_uint32), ("n_phases", ctypes.c_uint32),
        ("p_atomic_q32", ctypes.c_uint32), ("id_atomic", ctypes.c_uint32),
    ]


def mix64(z: int) -> int:
    """splitmix64 finalizer (same constants as tg_core.h)."""
    z = (z + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _u01(seed: int, a: int, b: int) -> float:
    """Uniform in (0, 1) from the counter hash (host-side parameter draws)."""
    return ((mix64(mix64(seed ^ (a * 0x9E37)) ^ b) >> 11) + 0.5) / float(1 << 53)


def q32(p: float) -> int:
    return max(0, min(Q32 - 1, int(math.floor(p * Q32))))


def zipf_cdf(n: int = N_COMPUTE_IDS, s: float = 1.2) -> np.ndarray:
    w = [1.0 / (r ** s) for r in range(1, n + 1)]
    tot = sum(w)
    out, acc = [], 0.0
    for x in w:
        acc += x
        out.append(q32(acc / tot))
    out[-1] = Q32 - 1
    return np.array(out, dtype=np.uint32)


def site_thresholds(n_sites: int, seed: int, dist: str) -> np.ndarray:
    """Per-site taken probability as a q32 threshold.

    'uniform' : p ~ U(0,1);  'beta05' : p ~ Beta(1/2, 1/2) = sin^2(pi u / 2).
    """
    out = np.empty(n_sites, dtype=np.uint32)
    for s in range(n_sites):
        u = _u01(seed, 0x5173, s)
        p = u if dist == "uniform" else math.sin(math.pi * u / 2.0) ** 2
        out[s] = q32(p)
    return out


def opcode_table() -> np.ndarray:
    """(op_class u16, simd_width u8, kind u8) per id as a structured array."""
    dt = np.dtype([("op_class", "<u2"), ("simd_width", "u1"), ("kind", "u1")])
    t = np.zeros(N_OPCODE_IDS, dtype=dt)
    for i in range(N_COMPUTE_IDS):
        # two width variants share one class: classes 0..29, widths 1,2,4,8,16
        t[i] = (i // 2, 1 << (i % 5), KIND_COMPUTE)
    t[ID_LOAD] = (30, 1, KIND_LOAD)
    t[ID_STORE] = (31, 1, KIND_STORE)
    t[ID_BRANCH] = (32, 1, KIND_BRANCH)
    t[ID_BARRIER] = (33, 1, KIND_BARRIER)
    t[ID_RET] = (34, 1, KIND_OTHER)
    t[ID_ATOMIC] = (35, 1, KIND_ATOMIC)
    return t


N_CLASSES = 36


@dataclass
class TraceSpec:
    """Parameters of one synthetic trace (see tg_core.h for the recipe)."""
    seed: int
    n_wi: int
    wg_size: int
    len_min: int
    len_max: int
    barrier_period: int = 256
    p_mem: float = 0.30
    p_branch: float = 0.05
    p_store: float = 0.5
    p_atomic: float = 0.0                 # share of memory instructions that are atomic RMWs
    p_local: float = 0.0
    mix: tuple = (1.0, 0.0, 0.0)          # global (sweep, stencil, random)
    sweep_base: int = 1 << 28
    sweep_stride: int = 4
    sweep_span: int = 1 << 19
    stencil_base: int = 0x20_0000_0000
    stencil_dim: int = 4096
    random_base: int = 1 << 28
    random_words: int = 1 << 17
    local_words: int = 1 << 14
    n_sites: int = 16
    site_dist: str = "uniform"
    history_len: int = 16
    label: str = ""

    def params(self) -> TgParams:
        p = TgParams()
        p.seed = self.seed & MASK64
        p.n_wi = self.n_wi
        p.wg_size = self.wg_size
        p.len_min, p.len_max = self.len_min, self.len_max
        p.barrier_period = self.barrier_period
        p.p_mem_q32 = q32(self.p_mem)
        p.p_branch_q32 = q32(self.p_branch)
        p.p_store_q32 = q32(self.p_store)
        p.p_local_q32 = q32(self.p_local) if self.p_local > 0 else 0
        tot = float(sum(self.mix))
        p.t_sweep_q32 = q32(self.mix[0] / tot)
        p.t_stencil_q32 = q32((self.mix[0] + self.mix[1]) / tot)
        p.sweep_base = self.sweep_base
        p.sweep_stride = self.sweep_stride
        p.sweep_words = max(1, self.sweep_span // self.sweep_stride)
        p.stencil_base = self.stencil_base
        p.stencil_dim = max(3, self.stencil_dim)
        p.random_base = self.random_base
        p.random_words = max(1, self.random_words)
        p.local_words = max(1, self.local_words)
        p.n_compute_ids = N_COMPUTE_IDS
        p.id_load, p.id_store, p.id_branch = ID_LOAD, ID_STORE, ID_BRANCH
        p.id_barrier, p.id_ret = ID_BARRIER, ID_RET
        p.n_sites = self.n_sites
        p.p_atomic_q32 = q32(self.p_atomic) if self.p_atomic > 0 else 0
        p.id_atomic = ID_ATOMIC
        return p

    def tables(self):
        return zipf_cdf(), site_thresholds(self.n_sites, self.seed, self.site_dist)


# ----------------------------------------------------------------- workloads
def config1(seed: int = 0) -> TraceSpec:
    """Plain single trace: 256 WIs (4 WGs of 64), ~2k events each, global
    4-byte accesses over a 512 KiB array (half stride-4 sequential, half
    uniform random), 16 branch sites with p ~ U(0,1), barrier every 256."""
    return TraceSpec(seed=seed, n_wi=256, wg_size=64, len_min=1536, len_max=2560,
                     mix=(0.5, 0.0, 0.5), sweep_base=1 << 28, sweep_stride=4,
                     sweep_span=1 << 19, random_base=1 << 28, random_words=1 << 17,
                     n_sites=16, site_dist="uniform", history_len=16, label="config1")


def _stride_for(seed: int) -> int:
    return 1 << (2 + mix64(seed ^ 0x57A1DE) % 7)   # 4 .. 256 bytes


def config2(seed: int = 1, n_wi: int = 1 << 20, len_min: int = 768,
            len_max: int = 1280) -> TraceSpec:
    """Plain large trace: 2^20 WIs in WGs of 256 (~1e9 events); 10% local
    accesses in a 64 KiB window; global 60/30/10 sweep (stride 4..256 B over
    1 GiB) / 5-point stencil on a 4096^2 float grid / uniform gather over
    1 GiB; 4096 sites with Beta(1/2,1/2) bias; history 16."""
    return TraceSpec(seed=seed, n_wi=n_wi, wg_size=256, len_min=len_min, len_max=len_max,
                     p_local=0.10, mix=(0.6, 0.3, 0.1),
                     sweep_base=0x10_0000_0000, sweep_stride=_stride_for(seed),
                     sweep_span=1 << 30, stencil_base=0x20_0000_0000, stencil_dim=4096,
                     random_base=0x30_0000_0000, random_words=1 << 28,
                     local_words=1 << 14, n_sites=4096, site_dist="beta05",
                     history_len=16, label="config2")


def config3_specs(seed: int = 2, n_traces: int = 512, scale: float = 1.0) -> List[TraceSpec]:
    """Batched: traces of log-uniform length 1e4..1e8 events (x scale), each
    with footprint 2^16..2^32 B and a Dirichlet(1,1,1) pattern mix."""
    out = []
    for i in range(n_traces):
        u = _u01(seed, 1, i)
        L = max(1024.0, round(10 ** (4 + 4 * u)) * scale)
        e = 16 + int(mix64(seed * 7919 + i) % 17)
        F = 1 << e
        g = [-math.log(_u01(seed, 10 + j, i)) for j in range(3)]
        stride = _stride_for(seed * 1_000_003 + i)
        G = max(3, int(math.isqrt(F // 4)))
        ts = TraceSpec(seed=seed * 100_000 + i, n_wi=max(1, math.ceil(L / 1024)),
                       wg_size=256, len_min=768, len_max=1280, p_local=0.10,
                       mix=tuple(g), sweep_base=0x10_0000_0000, sweep_stride=min(stride, F),
                       sweep_span=F, stencil_base=0x20_0000_0000, stencil_dim=G,
                       random_base=0x30_0000_0000, random_words=max(1, F // 4),
                       local_words=1 << 14, n_sites=4096, site_dist="beta05",
                       history_len=16, label=f"config3[{i}]")
        out.append(ts)
    return out


def config2_family(seed: int, n_traces: int, wi_log2_lo: float, wi_log2_hi: float,
                   len_min: int = 768, len_max: int = 1280) -> List[TraceSpec]:
    """Training/eval family for the sizing network: config-2 recipe with
    log-uniform work-item counts, per-trace stride and pattern mix."""
    out = []
    for i in range(n_traces):
        u = _u01(seed, 3, i)
        W = int(round(2 ** (wi_log2_lo + (wi_log2_hi - wi_log2_lo) * u)))
        g = [-math.log(_u01(seed, 20 + j, i)) for j in range(3)]
        ts = config2(seed=seed * 1_000_000 + i, n_wi=max(1, W), len_min=len_min, len_max=len_max)
        ts = replace(ts, mix=tuple(g), p_local=0.02 + 0.2 * _u01(seed, 30, i),
                     random_words=1 << (16 + int(mix64(seed + 31 * i) % 13)),
                     label=f"family{seed}[{i}]")
        out.append(ts)
    return out


def config5_specs(seed: int = 5, n_traces: int = 64, total_mem_log2: int = 32,
                  cap_log2: int = 28) -> List[TraceSpec]:
    """Stress: n_mem_i = 2^(20+8u) scaled to a total of 2^total_mem_log2,
    capped at 2^cap_log2 (excess water-filled); all global, uniform over
    1 GiB (2^28 words); 2^16 sites, Beta(1/2,1/2); history 32."""
    raw = [2 ** (20 + 8 * _u01(seed, 2, i)) for i in range(n_traces)]
    total = float(1 << total_mem_log2)
    cap = float(1 << cap_log2)
    w = [r * total / sum(raw) for r in raw]
    for _ in range(64):  # water-fill the excess over the cap
        over = sum(max(0.0, x - cap) for x in w)
        if over <= 0.5:
            break
        free = [i for i, x in enumerate(w) if x < cap]
        w = [min(x, cap) for x in w]
        fs = sum(w[i] for i in free)
        for i in free:
            w[i] += over * w[i] / fs
    out = []
    for i, nm in enumerate(w):
        n_ev = nm / 0.30
        n_wi = max(1, int(round(n_ev / 1024)))
        out.append(TraceSpec(seed=seed * 100_000 + i, n_wi=n_wi, wg_size=256, len_min=768,
                             len_max=1280, mix=(0.0, 0.0, 1.0), random_base=0x30_0000_0000,
                             random_words=1 << 28, n_sites=1 << 16, site_dist="beta05",
                             history_len=32, label=f"config5[{i}]"))
    return out


# -------------------------------------------------------------- generation
_host = None
_dev = None


def _load_host():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            raise RuntimeError(f"{HOST_LIB} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(HOST_LIB)
        L.tg_host_plan.restype = ctypes.c_void_p
        L.tg_host_plan.argtypes = [ctypes.POINTER(TgParams), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.tg_host_fill.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 5
        L.tg_host_wi_offsets.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.tg_host_free.argtypes = [ctypes.c_void_p]
        _host = L
    return _host


def _load_dev():
    global _dev
    if _dev is None:
        if not os.path.exists(DEV_LIB):
            raise RuntimeError(f"{DEV_LIB} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(DEV_LIB)
        L.tg_dev_plan.restype = ctypes.c_void_p
        L.tg_dev_plan.argtypes = [ctypes.POINTER(TgParams), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64)]
        L.tg_dev_fill.restype = ctypes.c_int
        L.tg_dev_fill.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        L.tg_dev_free.argtypes = [ctypes.c_void_p]
        _dev = L
    return _dev


@dataclass
class HostTrace:
    """A trace in host memory (numpy arrays)."""
    spec: TraceSpec
    opcode: np.ndarray
    wi_offsets: np.ndarray
    addr: np.ndarray
    mem_kind: np.ndarray
    br_site: np.ndarray
    br_taken: np.ndarray
    table: np.ndarray = field(default_factory=opcode_table)

    @property
    def n_sites(self) -> int:
        return self.spec.n_sites

    @property
    def history_len(self) -> int:
        return self.spec.history_len


def generate_host(spec: TraceSpec, threads: Optional[int] = None) -> HostTrace:
    L = _load_host()
    P = spec.params()
    zc, thr = spec.tables()
    ne, nm, nb = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    th = threads or min(16, os.cpu_count() or 1)
    plan = L.tg_host_plan(ctypes.byref(P), zc.ctypes.data, thr.ctypes.data, th,
                          ctypes.byref(ne), ctypes.byref(nm), ctypes.byref(nb))
    if not plan:
        raise ValueError("invalid trace parameters")
    try:
        op = np.empty(ne.value, dtype=np.uint16)
        off = np.empty(spec.n_wi + 1, dtype=np.uint64)
        addr = np.empty(nm.value, dtype=np.uint64)
        kind = np.empty(nm.value, dtype=np.uint8)
        site = np.empty(nb.value, dtype=np.uint32)
        taken = np.empty(nb.value, dtype=np.uint8)
        L.tg_host_wi_offsets(plan, off.ctypes.data)
        L.tg_host_fill(plan, th, op.ctypes.data, addr.ctypes.data, kind.ctypes.data,
                       site.ctypes.data, taken.ctypes.data)
    finally:
        L.tg_host_free(plan)
    return HostTrace(spec, op, off, addr, kind, site, taken)


def generate_device(spec: TraceSpec, device: int = 0) -> Dict[str, "object"]:
    """Generate straight into device memory; returns torch tensors."""
    import torch
    L = _load_dev()
    P = spec.params()
    zc, thr = spec.tables()
    ne, nm, nb = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    with torch.cuda.device(device):
        plan = L.tg_dev_plan(ctypes.byref(P), zc.ctypes.data, thr.ctypes.data,
                             ctypes.byref(ne), ctypes.byref(nm), ctypes.byref(nb))
        if not plan:
            raise RuntimeError("device trace plan failed")
        try:
            dev = torch.device("cuda", device)
            t = {
                "opcode": torch.empty(max(1, ne.value), dtype=torch.int16, device=dev),
                "wi_offsets": torch.empty(spec.n_wi + 1, dtype=torch.int64, device=dev),
                "addr": torch.empty(max(1, nm.value), dtype=torch.int64, device=dev),
                "mem_kind": torch.empty(max(1, nm.value), dtype=torch.uint8, device=dev),
                "br_site": torch.empty(max(1, nb.value), dtype=torch.int32, device=dev),
                "br_taken": torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev),
            }
            torch.cuda.synchronize(device)
            rc = L.tg_dev_fill(plan, t["wi_offsets"].data_ptr(), t["opcode"].data_ptr(),
                               t["addr"].data_ptr(), t["mem_kind"].data_ptr(),
                               t["br_site"].data_ptr(), t["br_taken"].data_ptr())
            if rc != 0:
                raise RuntimeError(f"device trace fill failed ({rc})")
        finally:
            L.tg_dev_free(plan)
    t["n_events"], t["n_mem"], t["n_branch"] = ne.value, nm.value, nb.value
    t["spec"] = spec
    return t
