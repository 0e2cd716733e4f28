"""Kernel programs for the trace producer, and their seeded inputs.

A program is a list of 24-byte instruction records (the aiwc_insn layout of
the library's header) plus the opcode table its ids index.  ``Asm`` encodes
them: each operation gets the LLVM opcode name the paper's tool would see
for it (the opcode metrics count LLVM opcode names: Implementation section),
and each conditional branch gets its own site.  The assembler only encodes;
running a program is the producer's job (the GPU library) and the oracle's.

The kernels follow dwarfs of the paper's workload suite in shape -- a
dense map, a structured-grid stencil, a tree reduction in local memory,
histograms with global and local atomics, a CSR sparse matrix-vector
product, a bitwise CRC, a tiled matrix product in local memory, and a
Needleman-Wunsch wavefront with a barrier per anti-diagonal.  Each builder
returns a ``Launch``: program, ND-range, arguments (numpy buffers, local
sizes, scalars) drawn from a seeded generator.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

INSN_DTYPE = np.dtype([("op", "u1"), ("mode", "u1"), ("width", "u1"), ("flags", "u1"),
                       ("d", "u1"), ("a", "u1"), ("b", "u1"), ("c", "u1"), ("id", "<u2"),
                       ("site", "<u2"), ("target2", "<u4"), ("imm", "<i8")])
assert INSN_DTYPE.itemsize == 24
TABLE_DTYPE = np.dtype([("op_class", "<u2"), ("simd_width", "u1"), ("kind", "u1")])

# operation numbers (aiwc_insn.op)
(RET, MOV, ADD, SUB, MUL, SDIV, SREM, UDIV, UREM, SHL, LSHR, ASHR, AND, OR, XOR, ICMP, FADD,
 FSUB, FMUL, FDIV, FCMP, FMA, FSQRT, FMIN, FMAX, SITOFP, FPTOSI, SEXT, ZEXT, SELECT, GEP, LOAD,
 STORE, ATOMIC, BR, JMP, BARRIER, BUILTIN) = range(38)
# opcode kinds
K_COMPUTE, K_LOAD, K_STORE, K_ATOMIC, K_BRANCH, K_BARRIER, K_OTHER = range(7)
ICMP_PRED = {"eq": 0, "ne": 1, "slt": 2, "sle": 3, "sgt": 4, "sge": 5, "ult": 6, "ule": 7,
             "ugt": 8, "uge": 9}
FCMP_PRED = {"oeq": 0, "une": 1, "olt": 2, "ole": 3, "ogt": 4, "oge": 5}
LOAD_MODE = {"i32": 0, "u32": 1, "f32": 1, "64": 2}
ATOMIC_MODE = {"add": 0, "sub": 1, "and": 2, "or": 3, "xor": 4, "min": 5, "max": 6, "umin": 7,
               "umax": 8}
BUILTIN_MODE = {"global_id": 0, "local_id": 3, "group_id": 6, "global_size": 9,
                "local_size": 12, "num_groups": 15}
IMM_B = 1
ADDR_TAG_SHIFT = 40

# LLVM opcode name and kind of each operation
_NAME = {RET: "ret", MOV: "phi", ADD: "add", SUB: "sub", MUL: "mul", SDIV: "sdiv", SREM: "srem",
         UDIV: "udiv", UREM: "urem", SHL: "shl", LSHR: "lshr", ASHR: "ashr", AND: "and", OR: "or",
         XOR: "xor", ICMP: "icmp", FADD: "fadd", FSUB: "fsub", FMUL: "fmul", FDIV: "fdiv",
         FCMP: "fcmp", FMA: "call", FSQRT: "call", FMIN: "call", FMAX: "call", SITOFP: "sitofp",
         FPTOSI: "fptosi", SEXT: "sext", ZEXT: "zext", SELECT: "select", GEP: "getelementptr",
         LOAD: "load", STORE: "store", ATOMIC: "atomicrmw", BR: "br", JMP: "br", BARRIER: "call",
         BUILTIN: "call"}
_ARITH = {ADD, SUB, MUL, SDIV, SREM, UDIV, UREM, SHL, LSHR, ASHR, AND, OR, XOR, ICMP, FADD, FSUB,
          FMUL, FDIV, FCMP, FMA, FSQRT, FMIN, FMAX, SELECT}
_KIND = {LOAD: K_LOAD, STORE: K_STORE, ATOMIC: K_ATOMIC, BR: K_BRANCH, BARRIER: K_BARRIER}


def f32_bits(x: float) -> int:
    return struct.unpack("<I", struct.pack("<f", x))[0]


# kernel arguments (kind numbers = aiwc_kernel_arg.kind)
@dataclass
class Global:
    array: np.ndarray
    kind: int = 0


@dataclass
class Local:
    nbytes: int
    kind: int = 1


@dataclass
class Scalar:
    value: int
    kind: int = 2


@dataclass
class Program:
    name: str
    code: np.ndarray          # INSN_DTYPE
    table: np.ndarray         # TABLE_DTYPE
    n_sites: int
    class_names: List[str]
    id_names: List[str]       # LLVM name of each opcode id


@dataclass
class Launch:
    program: Program
    global_size: Tuple[int, ...]
    local_size: Tuple[int, ...]
    args: List
    expected: Dict[str, np.ndarray] = field(default_factory=dict)  # buffer name -> result
    names: Dict[str, int] = field(default_factory=dict)             # buffer name -> arg index

    def fresh_args(self) -> List:
        """Copies of the arguments (global buffers copied)."""
        return [Global(a.array.copy()) if isinstance(a, Global) else a for a in self.args]


class Asm:
    """Builds a program.  Registers are ints 0..63; r0.. hold the arguments.
    Operand `b` may be an int register or, via imm=..., an immediate."""

    def __init__(self, name: str):
        self.name = name
        self.rows: List[dict] = []
        self.labels: Dict[str, int] = {}
        self.ids: Dict[Tuple[str, int, int], int] = {}
        self.classes: Dict[str, int] = {}
        self.n_sites = 0

    def _id(self, op: int, width: int) -> int:
        name = _NAME[op]
        kind = _KIND.get(op, K_COMPUTE if op in _ARITH else K_OTHER)
        simd = 1 if op in (STORE, BR, JMP, BARRIER, RET) else width
        key = (name, simd, kind)
        if key not in self.ids:
            self.classes.setdefault(name, len(self.classes))
            self.ids[key] = len(self.ids)
        return self.ids[key]

    def emit(self, op, d=0, a=0, b=0, c=0, imm=None, mode=0, width=1, target=None, target2=None):
        row = dict(op=op, mode=mode, width=width, flags=0, d=d, a=a, b=b, c=c,
                   id=self._id(op, width), site=0, target2=0, imm=0, t1=target, t2=target2)
        if imm is not None:
            row["imm"] = int(imm)
            if op not in (GEP, BR, JMP):
                row["flags"] = IMM_B
        if op == BR:
            row["site"] = self.n_sites
            self.n_sites += 1
        self.rows.append(row)

    def label(self, name: str):
        assert name not in self.labels
        self.labels[name] = len(self.rows)

    # -- integer
    def _bin(self, op, d, a, b, width=1):
        if isinstance(b, Imm):
            self.emit(op, d=d, a=a, imm=b.v, width=width)
        else:
            self.emit(op, d=d, a=a, b=b, width=width)

    def mov(self, d, b, width=1):
        if isinstance(b, Imm):
            self.emit(MOV, d=d, imm=b.v, width=width)
        else:
            self.emit(MOV, d=d, b=b, width=width)

    def add(self, d, a, b, width=1): self._bin(ADD, d, a, b, width)
    def sub(self, d, a, b, width=1): self._bin(SUB, d, a, b, width)
    def mul(self, d, a, b, width=1): self._bin(MUL, d, a, b, width)
    def sdiv(self, d, a, b): self._bin(SDIV, d, a, b)
    def srem(self, d, a, b): self._bin(SREM, d, a, b)
    def udiv(self, d, a, b): self._bin(UDIV, d, a, b)
    def urem(self, d, a, b): self._bin(UREM, d, a, b)
    def shl(self, d, a, b): self._bin(SHL, d, a, b)
    def lshr(self, d, a, b): self._bin(LSHR, d, a, b)
    def ashr(self, d, a, b): self._bin(ASHR, d, a, b)
    def and_(self, d, a, b): self._bin(AND, d, a, b)
    def or_(self, d, a, b): self._bin(OR, d, a, b)
    def xor(self, d, a, b): self._bin(XOR, d, a, b)

    def icmp(self, pred, d, a, b, width=1):
        m = ICMP_PRED[pred]
        if isinstance(b, Imm):
            self.emit(ICMP, d=d, a=a, imm=b.v, mode=m, width=width)
        else:
            self.emit(ICMP, d=d, a=a, b=b, mode=m, width=width)

    # -- binary32
    def fadd(self, d, a, b, width=1): self._bin(FADD, d, a, b, width)
    def fsub(self, d, a, b, width=1): self._bin(FSUB, d, a, b, width)
    def fmul(self, d, a, b, width=1): self._bin(FMUL, d, a, b, width)
    def fdiv(self, d, a, b, width=1): self._bin(FDIV, d, a, b, width)
    def fmin(self, d, a, b, width=1): self._bin(FMIN, d, a, b, width)
    def fmax(self, d, a, b, width=1): self._bin(FMAX, d, a, b, width)

    def fcmp(self, pred, d, a, b, width=1):
        m = FCMP_PRED[pred]
        if isinstance(b, Imm):
            self.emit(FCMP, d=d, a=a, imm=b.v, mode=m, width=width)
        else:
            self.emit(FCMP, d=d, a=a, b=b, mode=m, width=width)

    def fma(self, d, a, b, c, width=1): self.emit(FMA, d=d, a=a, b=b, c=c, width=width)
    def fsqrt(self, d, a, width=1): self.emit(FSQRT, d=d, a=a, width=width)
    def sitofp(self, d, a, width=1): self.emit(SITOFP, d=d, a=a, width=width)
    def fptosi(self, d, a, width=1): self.emit(FPTOSI, d=d, a=a, width=width)
    def sext(self, d, a, width=1): self.emit(SEXT, d=d, a=a, width=width)
    def zext(self, d, a, width=1): self.emit(ZEXT, d=d, a=a, width=width)

    def select(self, d, cond, b, c, width=1):
        if isinstance(b, Imm):
            self.emit(SELECT, d=d, a=cond, imm=b.v, c=c, width=width)
        else:
            self.emit(SELECT, d=d, a=cond, b=b, c=c, width=width)

    # -- memory
    def gep(self, d, base, index=None, scale=1, offset=None):
        """d = base + index * scale, or d = base + offset."""
        if index is None:
            self.emit(GEP, d=d, a=base, imm=offset)
            self.rows[-1]["flags"] = IMM_B
        else:
            self.emit(GEP, d=d, a=base, b=index, imm=scale)

    def load(self, d, addr, ty="u32", width=1):
        self.emit(LOAD, d=d, a=addr, mode=LOAD_MODE[ty], width=width)

    def store(self, addr, b, size=4, width=1):
        m = 1 if size == 8 else 0
        if isinstance(b, Imm):
            self.emit(STORE, a=addr, imm=b.v, mode=m, width=width)
        else:
            self.emit(STORE, a=addr, b=b, mode=m, width=width)

    def atomic(self, op, d, addr, b):
        m = ATOMIC_MODE[op]
        if isinstance(b, Imm):
            self.emit(ATOMIC, d=d, a=addr, imm=b.v, mode=m)
        else:
            self.emit(ATOMIC, d=d, a=addr, b=b, mode=m)

    # -- control
    def br(self, cond, t: str, f: str):
        self.emit(BR, a=cond, target=t, target2=f)

    def jmp(self, t: str):
        self.emit(JMP, target=t)

    def barrier(self):
        self.emit(BARRIER)

    def builtin(self, fn: str, d, dim=0):
        self.emit(BUILTIN, d=d, mode=BUILTIN_MODE[fn] + dim)

    def ret(self):
        self.emit(RET)

    def finish(self) -> Program:
        code = np.zeros(len(self.rows), dtype=INSN_DTYPE)
        for i, r in enumerate(self.rows):
            for k in ("op", "mode", "width", "flags", "d", "a", "b", "c", "id", "site", "imm"):
                code[i][k] = r[k]
            if r["t1"] is not None:
                code[i]["imm"] = self.labels[r["t1"]]
            if r["t2"] is not None:
                code[i]["target2"] = self.labels[r["t2"]]
        table = np.zeros(len(self.ids), dtype=TABLE_DTYPE)
        id_names = [""] * len(self.ids)
        for (name, simd, kind), i in self.ids.items():
            table[i] = (self.classes[name], simd, kind)
            id_names[i] = name
        class_names = [""] * len(self.classes)
        for name, i in self.classes.items():
            class_names[i] = name
        return Program(self.name, code, table, self.n_sites, class_names, id_names)


@dataclass(frozen=True)
class Imm:
    v: int


def I(v: int) -> Imm:
    return Imm(int(v))


def F(x: float) -> Imm:
    return Imm(f32_bits(x))


# ----------------------------------------------------------------- kernels

def vector_add(n: int, wg: int = 256, seed: int = 0) -> Launch:
    """c[i] = a[i] + b[i] for i < n; the range is rounded up to the group size."""
    A = Asm("vector_add")
    A.builtin("global_id", 4)
    A.icmp("ult", 5, 4, 3)
    A.br(5, "body", "end")
    A.label("body")
    A.gep(6, 0, 4, 4); A.load(7, 6, "f32")
    A.gep(6, 1, 4, 4); A.load(8, 6, "f32")
    A.fadd(9, 7, 8)
    A.gep(6, 2, 4, 4); A.store(6, 9)
    A.label("end")
    A.ret()
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    c = np.zeros(n, dtype=np.float32)
    g = -(-n // wg) * wg
    return Launch(A.finish(), (g,), (wg,), [Global(a), Global(b), Global(c), Scalar(n)],
                  expected={"c": a + b}, names={"c": 2})


def vector_add4(n4: int, wg: int = 64, seed: int = 0) -> Launch:
    """The same map on 4-wide vectors: one work-item adds a float4."""
    A = Asm("vector_add4")
    A.builtin("global_id", 4)
    A.icmp("ult", 5, 4, 3)
    A.br(5, "body", "end")
    A.label("body")
    A.gep(6, 0, 4, 16); A.load(8, 6, "f32", width=4)
    A.gep(6, 1, 4, 16); A.load(12, 6, "f32", width=4)
    A.fadd(16, 8, 12, width=4)
    A.gep(6, 2, 4, 16); A.store(6, 16, width=4)
    A.label("end")
    A.ret()
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(4 * n4).astype(np.float32)
    b = rng.standard_normal(4 * n4).astype(np.float32)
    c = np.zeros(4 * n4, dtype=np.float32)
    g = -(-n4 // wg) * wg
    return Launch(A.finish(), (g,), (wg,), [Global(a), Global(b), Global(c), Scalar(n4)],
                  expected={"c": a + b}, names={"c": 2})


def stencil2d(nx: int, ny: int, lx: int = 16, ly: int = 16, seed: int = 0) -> Launch:
    """Structured grid: interior points relax toward the mean of their four
    neighbours, boundary points copy.  The interior test is four
    short-circuit branches, as a compiler lowers `a && b && c && d`."""
    A = Asm("stencil2d")
    A.builtin("global_id", 4, 0)
    A.builtin("global_id", 5, 1)
    A.mul(6, 5, 2); A.add(6, 6, 4)
    A.gep(7, 0, 6, 4); A.load(8, 7, "f32")
    A.icmp("ugt", 9, 4, I(0)); A.br(9, "c2", "edge")
    A.label("c2"); A.sub(10, 2, I(1)); A.icmp("ult", 9, 4, 10); A.br(9, "c3", "edge")
    A.label("c3"); A.icmp("ugt", 9, 5, I(0)); A.br(9, "c4", "edge")
    A.label("c4"); A.sub(10, 3, I(1)); A.icmp("ult", 9, 5, 10); A.br(9, "inner", "edge")
    A.label("inner")
    A.gep(11, 7, offset=-4); A.load(12, 11, "f32")
    A.gep(11, 7, offset=4); A.load(13, 11, "f32")
    A.sub(14, 6, 2); A.gep(11, 0, 14, 4); A.load(15, 11, "f32")
    A.add(14, 6, 2); A.gep(11, 0, 14, 4); A.load(16, 11, "f32")
    A.fadd(17, 12, 13); A.fadd(17, 17, 15); A.fadd(17, 17, 16)
    A.fmul(17, 17, F(0.25))
    A.fsub(18, 17, 8); A.fmul(18, 18, F(0.5)); A.fadd(18, 8, 18)
    A.gep(11, 1, 6, 4); A.store(11, 18); A.jmp("end")
    A.label("edge")
    A.gep(11, 1, 6, 4); A.store(11, 8)
    A.label("end")
    A.ret()
    rng = np.random.default_rng(seed)
    src = rng.standard_normal((ny, nx)).astype(np.float32)
    out = np.zeros_like(src)
    exp = src.copy()
    if nx > 2 and ny > 2:
        c = src[1:-1, 1:-1]
        s = ((src[1:-1, :-2] + src[1:-1, 2:]) + src[:-2, 1:-1]) + src[2:, 1:-1]
        s = s * np.float32(0.25)
        exp[1:-1, 1:-1] = c + (s - c) * np.float32(0.5)
    return Launch(A.finish(), (nx, ny), (lx, ly),
                  [Global(src.ravel()), Global(out.ravel()), Scalar(nx), Scalar(ny)],
                  expected={"out": exp.ravel()}, names={"out": 1})


def reduce_local(n: int, wg: int = 256, seed: int = 0) -> Launch:
    """Per-work-group int32 sums: a tree in local memory, a barrier per level."""
    A = Asm("reduce_local")
    A.builtin("global_id", 4); A.builtin("local_id", 5); A.builtin("local_size", 6)
    A.mov(7, I(0))
    A.icmp("ult", 8, 4, 3); A.br(8, "ld", "st")
    A.label("ld"); A.gep(9, 0, 4, 4); A.load(7, 9, "i32")
    A.label("st"); A.gep(10, 2, 5, 4); A.store(10, 7)
    A.barrier()
    A.lshr(11, 6, I(1))
    A.label("loop"); A.icmp("ugt", 8, 11, I(0)); A.br(8, "body", "done")
    A.label("body"); A.icmp("ult", 8, 5, 11); A.br(8, "add", "sync")
    A.label("add")
    A.add(12, 5, 11); A.gep(13, 2, 12, 4); A.load(14, 13, "i32"); A.load(15, 10, "i32")
    A.add(15, 15, 14); A.store(10, 15)
    A.label("sync"); A.barrier(); A.lshr(11, 11, I(1)); A.jmp("loop")
    A.label("done"); A.icmp("eq", 8, 5, I(0)); A.br(8, "wr", "end")
    A.label("wr"); A.builtin("group_id", 16); A.load(15, 10, "i32"); A.gep(13, 1, 16, 4); A.store(13, 15)
    A.label("end"); A.ret()
    rng = np.random.default_rng(seed)
    g = -(-n // wg) * wg
    x = rng.integers(-1000, 1000, n, dtype=np.int32)
    out = np.zeros(g // wg, dtype=np.int32)
    pad = np.zeros(g, dtype=np.int64)
    pad[:n] = x
    exp = pad.reshape(-1, wg).sum(axis=1).astype(np.int32)
    return Launch(A.finish(), (g,), (wg,),
                  [Global(x), Global(out), Local(4 * wg), Scalar(n)],
                  expected={"out": exp}, names={"out": 1})


def histogram(n: int, nbins: int, n_wi: int = 4096, wg: int = 256, seed: int = 0,
              zipf: float = 0.0) -> Launch:
    """Grid-stride histogram with one global atomic add per element."""
    A = Asm("histogram")
    A.builtin("global_id", 4); A.builtin("global_size", 5)
    A.label("loop"); A.icmp("ult", 6, 4, 2); A.br(6, "body", "end")
    A.label("body")
    A.gep(7, 0, 4, 4); A.load(8, 7, "u32"); A.urem(9, 8, 3); A.gep(10, 1, 9, 4)
    A.atomic("add", 11, 10, I(1)); A.add(4, 4, 5); A.jmp("loop")
    A.label("end"); A.ret()
    data = _hist_data(n, nbins, seed, zipf)
    hist = np.zeros(nbins, dtype=np.uint32)
    return Launch(A.finish(), (n_wi,), (wg,), [Global(data), Global(hist), Scalar(n), Scalar(nbins)],
                  expected={"hist": np.bincount(data % nbins, minlength=nbins).astype(np.uint32)},
                  names={"hist": 1})


def histogram_local(n: int, nbins: int, n_wi: int = 4096, wg: int = 256, seed: int = 0,
                    zipf: float = 0.0) -> Launch:
    """Privatised histogram: local atomics, a barrier, then one global atomic
    per bin and work-group."""
    A = Asm("histogram_local")
    A.builtin("global_id", 5); A.builtin("global_size", 6)
    A.builtin("local_id", 7); A.builtin("local_size", 8)
    A.mov(15, 7)
    A.label("zl"); A.icmp("ult", 9, 15, 4); A.br(9, "zb", "zd")
    A.label("zb"); A.gep(13, 2, 15, 4); A.store(13, I(0)); A.add(15, 15, 8); A.jmp("zl")
    A.label("zd"); A.barrier()
    A.label("loop"); A.icmp("ult", 9, 5, 3); A.br(9, "body", "merge")
    A.label("body")
    A.gep(10, 0, 5, 4); A.load(11, 10, "u32"); A.urem(12, 11, 4); A.gep(13, 2, 12, 4)
    A.atomic("add", 14, 13, I(1)); A.add(5, 5, 6); A.jmp("loop")
    A.label("merge"); A.barrier(); A.mov(15, 7)
    A.label("ml"); A.icmp("ult", 9, 15, 4); A.br(9, "mb", "end")
    A.label("mb")
    A.gep(13, 2, 15, 4); A.load(16, 13, "u32"); A.gep(17, 1, 15, 4)
    A.atomic("add", 14, 17, 16); A.add(15, 15, 8); A.jmp("ml")
    A.label("end"); A.ret()
    data = _hist_data(n, nbins, seed, zipf)
    hist = np.zeros(nbins, dtype=np.uint32)
    return Launch(A.finish(), (n_wi,), (wg,),
                  [Global(data), Global(hist), Local(4 * nbins), Scalar(n), Scalar(nbins)],
                  expected={"hist": np.bincount(data % nbins, minlength=nbins).astype(np.uint32)},
                  names={"hist": 1})


def _hist_data(n, nbins, seed, zipf):
    rng = np.random.default_rng(seed)
    if zipf > 0:
        return (rng.zipf(1.0 + zipf, n) % (4 * nbins)).astype(np.uint32)
    return rng.integers(0, 1 << 31, n, dtype=np.int64).astype(np.uint32)


def csr_spmv(nrows: int, ncols: int, avg_nnz: float = 8.0, wg: int = 64, seed: int = 0) -> Launch:
    """y = A x with A in CSR, one work-item per row.  Values are small
    integers, so every sum is exact in binary32 whatever its order."""
    A = Asm("csr_spmv")
    A.builtin("global_id", 6); A.icmp("ult", 7, 6, 5); A.br(7, "row", "end")
    A.label("row")
    A.gep(8, 0, 6, 4); A.load(9, 8, "i32"); A.gep(8, 8, offset=4); A.load(10, 8, "i32")
    A.mov(11, F(0.0))
    A.label("loop"); A.icmp("slt", 7, 9, 10); A.br(7, "body", "fin")
    A.label("body")
    A.gep(12, 1, 9, 4); A.load(13, 12, "i32"); A.gep(12, 2, 9, 4); A.load(14, 12, "f32")
    A.gep(12, 3, 13, 4); A.load(15, 12, "f32"); A.fmul(16, 14, 15); A.fadd(11, 11, 16)
    A.add(9, 9, I(1)); A.jmp("loop")
    A.label("fin"); A.gep(12, 4, 6, 4); A.store(12, 11)
    A.label("end"); A.ret()
    rng = np.random.default_rng(seed)
    deg = rng.poisson(avg_nnz, nrows).astype(np.int64)
    rowptr = np.zeros(nrows + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(deg)
    nnz = int(rowptr[-1])
    col = rng.integers(0, ncols, nnz, dtype=np.int64).astype(np.int32)
    val = rng.integers(-4, 5, nnz).astype(np.float32)
    x = rng.integers(-4, 5, ncols).astype(np.float32)
    y = np.zeros(nrows, dtype=np.float32)
    exp = np.zeros(nrows, dtype=np.float64)
    np.add.at(exp, np.repeat(np.arange(nrows), deg), val.astype(np.float64) * x[col])
    g = -(-nrows // wg) * wg
    return Launch(A.finish(), (g,), (wg,),
                  [Global(rowptr), Global(col if nnz else np.zeros(1, np.int32)),
                   Global(val if nnz else np.zeros(1, np.float32)), Global(x), Global(y),
                   Scalar(nrows)],
                  expected={"y": exp.astype(np.float32)}, names={"y": 4})


def crc32(n_wi: int, words: int, wg: int = 64, seed: int = 0) -> Launch:
    """Bitwise reflected CRC-32 of each work-item's words (one data-dependent
    branch per bit)."""
    A = Asm("crc32")
    A.builtin("global_id", 3); A.mul(4, 3, 2); A.add(5, 4, 2); A.mov(6, I(0xFFFFFFFF))
    A.label("wloop"); A.icmp("ult", 7, 4, 5); A.br(7, "wbody", "fin")
    A.label("wbody"); A.gep(8, 0, 4, 4); A.load(9, 8, "u32"); A.xor(6, 6, 9); A.mov(10, I(32))
    A.label("bloop"); A.and_(11, 6, I(1)); A.br(11, "odd", "even")
    A.label("odd"); A.lshr(6, 6, I(1)); A.xor(6, 6, I(0xEDB88320)); A.jmp("bnext")
    A.label("even"); A.lshr(6, 6, I(1))
    A.label("bnext"); A.sub(10, 10, I(1)); A.icmp("ne", 7, 10, I(0)); A.br(7, "bloop", "wnext")
    A.label("wnext"); A.add(4, 4, I(1)); A.jmp("wloop")
    A.label("fin"); A.xor(6, 6, I(0xFFFFFFFF)); A.gep(8, 1, 3, 4); A.store(8, 6); A.ret()
    import zlib
    rng = np.random.default_rng(seed)
    data = rng.integers(0, 1 << 32, n_wi * words, dtype=np.uint64).astype(np.uint32)
    out = np.zeros(n_wi, dtype=np.uint32)
    exp = np.array([zlib.crc32(data[w * words:(w + 1) * words].astype("<u4").tobytes())
                    for w in range(n_wi)], dtype=np.uint32)
    return Launch(A.finish(), (n_wi,), (wg,), [Global(data), Global(out), Scalar(words)],
                  expected={"out": exp}, names={"out": 1})


def matmul_tiled(n: int, tile: int = 16, seed: int = 0) -> Launch:
    """C = A B with tile x tile work-groups staging tiles in local memory
    (two barriers per tile step).  Small-integer values keep every sum exact."""
    T = tile
    A = Asm("matmul_tiled")
    A.builtin("local_id", 6, 0); A.builtin("local_id", 7, 1)
    A.builtin("global_id", 8, 0); A.builtin("global_id", 9, 1)
    A.mov(10, F(0.0)); A.mov(11, I(0))
    A.mul(12, 7, I(T)); A.add(12, 12, 6); A.gep(13, 3, 12, 4); A.gep(14, 4, 12, 4)
    A.label("tloop"); A.icmp("ult", 15, 11, 5); A.br(15, "tbody", "fin")
    A.label("tbody")
    A.mul(16, 9, 5); A.add(16, 16, 11); A.add(16, 16, 6); A.gep(17, 0, 16, 4); A.load(18, 17, "f32")
    A.store(13, 18)
    A.add(16, 11, 7); A.mul(16, 16, 5); A.add(16, 16, 8); A.gep(17, 1, 16, 4); A.load(18, 17, "f32")
    A.store(14, 18)
    A.barrier()
    A.mov(19, I(0))
    A.label("kloop"); A.icmp("ult", 15, 19, I(T)); A.br(15, "kbody", "kdone")
    A.label("kbody")
    A.mul(20, 7, I(T)); A.add(20, 20, 19); A.gep(21, 3, 20, 4); A.load(22, 21, "f32")
    A.mul(20, 19, I(T)); A.add(20, 20, 6); A.gep(21, 4, 20, 4); A.load(23, 21, "f32")
    A.fmul(24, 22, 23); A.fadd(10, 10, 24); A.add(19, 19, I(1)); A.jmp("kloop")
    A.label("kdone"); A.barrier(); A.add(11, 11, I(T)); A.jmp("tloop")
    A.label("fin"); A.mul(16, 9, 5); A.add(16, 16, 8); A.gep(17, 2, 16, 4); A.store(17, 10); A.ret()
    assert n % T == 0
    rng = np.random.default_rng(seed)
    a = rng.integers(-3, 4, (n, n)).astype(np.float32)
    b = rng.integers(-3, 4, (n, n)).astype(np.float32)
    c = np.zeros((n, n), dtype=np.float32)
    exp = (a.astype(np.float64) @ b.astype(np.float64)).astype(np.float32)
    return Launch(A.finish(), (n, n), (T, T),
                  [Global(a.ravel()), Global(b.ravel()), Global(c.ravel()), Local(4 * T * T),
                   Local(4 * T * T), Scalar(n)],
                  expected={"c": exp.ravel()}, names={"c": 2})


def needle(n_tiles: int, B: int = 16, penalty: int = 10, seed: int = 0) -> Launch:
    """Needleman-Wunsch: each work-group fills one B x B score tile from its
    top row and left column, one anti-diagonal per barrier interval."""
    A = Asm("needle")
    A.builtin("local_id", 6); A.builtin("group_id", 7); A.builtin("local_size", 8); A.add(9, 8, I(1))
    A.mul(10, 7, 9); A.add(11, 10, 6); A.add(11, 11, I(1))
    A.gep(12, 1, 11, 4); A.load(13, 12, "i32"); A.add(14, 6, I(1)); A.gep(15, 4, 14, 4); A.store(15, 13)
    A.gep(12, 2, 11, 4); A.load(13, 12, "i32"); A.mul(14, 14, 9); A.gep(15, 4, 14, 4); A.store(15, 13)
    A.icmp("eq", 16, 6, I(0)); A.br(16, "corner", "sync0")
    A.label("corner"); A.gep(12, 1, 10, 4); A.load(13, 12, "i32"); A.store(4, 13)
    A.label("sync0"); A.barrier()
    A.mov(17, I(0)); A.add(18, 8, 8); A.sub(18, 18, I(1))
    A.label("dloop"); A.icmp("ult", 16, 17, 18); A.br(16, "dbody", "wout")
    A.label("dbody"); A.sub(19, 17, 6); A.icmp("ult", 16, 19, 8); A.br(16, "cell", "dsync")
    A.label("cell")
    A.add(20, 19, I(1)); A.mul(20, 20, 9); A.add(20, 20, 6); A.add(20, 20, I(1))
    A.sub(21, 20, 9); A.sub(21, 21, I(1)); A.gep(22, 4, 21, 4); A.load(23, 22, "i32")
    A.mul(24, 7, 8); A.mul(24, 24, 8); A.mul(25, 19, 8); A.add(24, 24, 25); A.add(24, 24, 6)
    A.gep(22, 0, 24, 4); A.load(25, 22, "i32"); A.add(23, 23, 25)
    A.add(21, 21, I(1)); A.gep(22, 4, 21, 4); A.load(26, 22, "i32"); A.sub(26, 26, 5)
    A.sub(21, 20, I(1)); A.gep(22, 4, 21, 4); A.load(27, 22, "i32"); A.sub(27, 27, 5)
    A.icmp("sgt", 16, 26, 23); A.select(23, 16, 26, 23)
    A.icmp("sgt", 16, 27, 23); A.select(23, 16, 27, 23)
    A.gep(22, 4, 20, 4); A.store(22, 23)
    A.gep(22, 3, 24, 4); A.store(22, 23)
    A.label("dsync"); A.barrier(); A.add(17, 17, I(1)); A.jmp("dloop")
    A.label("wout"); A.ret()
    rng = np.random.default_rng(seed)
    sim = rng.integers(-5, 6, (n_tiles, B, B)).astype(np.int32)
    top = rng.integers(-50, 50, (n_tiles, B + 1)).astype(np.int32)
    left = rng.integers(-50, 50, (n_tiles, B + 1)).astype(np.int32)
    left[:, 0] = top[:, 0]
    out = np.zeros((n_tiles, B, B), dtype=np.int32)
    exp = np.zeros_like(out)
    for t in range(n_tiles):
        S = np.zeros((B + 1, B + 1), dtype=np.int64)
        S[0, :] = top[t]
        S[1:, 0] = left[t, 1:]
        for i in range(1, B + 1):
            for j in range(1, B + 1):
                S[i, j] = max(S[i - 1, j - 1] + sim[t, i - 1, j - 1], S[i - 1, j] - penalty,
                              S[i, j - 1] - penalty)
        exp[t] = S[1:, 1:]
    return Launch(A.finish(), (n_tiles * B,), (B,),
                  [Global(sim.ravel()), Global(top.ravel()), Global(left.ravel()), Global(out.ravel()),
                   Local(4 * (B + 1) * (B + 1)), Scalar(penalty)],
                  expected={"out": exp.ravel()}, names={"out": 3})


def suite(scale: int = 1, seed: int = 0) -> List[Launch]:
    """One launch of every kernel; scale multiplies the problem sizes."""
    s = scale
    return [
        vector_add(1000 * s + 37, seed=seed),
        vector_add4(512 * s + 5, seed=seed + 1),
        stencil2d(48 * s, 32 * s, seed=seed + 2),
        reduce_local(3000 * s + 11, wg=128, seed=seed + 3),
        histogram(20000 * s, 97, n_wi=1024 * s, seed=seed + 4, zipf=0.5),
        histogram_local(20000 * s, 64, n_wi=1024 * s, wg=128, seed=seed + 5),
        csr_spmv(700 * s, 900 * s, seed=seed + 6),
        crc32(256 * s, 6, seed=seed + 7),
        matmul_tiled(32 * s, seed=seed + 8),
        needle(4 * s, B=16, seed=seed + 9),
    ]


FLOAT_OPS = ("fadd", "fsub", "fmul", "fdiv", "fma", "fsqrt", "fmin", "fmax", "sitofp", "fptosi",
             "fcmp_olt", "fcmp_une", "sdiv", "srem", "udiv", "urem", "ashr", "shl", "sext", "zext",
             "select")


def special_f32(n: int, seed: int = 0) -> np.ndarray:
    """binary32 values with NaNs, infinities, signed zeros, subnormals,
    integers at the int32 limits and ordinary numbers."""
    rng = np.random.default_rng(seed)
    pool = np.array([0.0, -0.0, 1.0, -1.0, 0.5, 3.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45,
                     1e-40, 1.17549435e-38, 3.4028235e38, -3.4028235e38, 2147483648.0,
                     -2147483648.0, 2147483520.0, -2147483904.0, 7.0, 1e-20, 123456.78],
                    dtype=np.float32)
    v = rng.standard_normal(n).astype(np.float32) * np.float32(100)
    pick = rng.random(n) < 0.6
    v[pick] = pool[rng.integers(0, pool.size, int(pick.sum()))]
    bits = v.view(np.uint32).copy()
    nan_payload = rng.random(n) < 0.05          # NaNs with other payloads and signs
    bits[nan_payload] = (0x7F800001 + rng.integers(0, 1 << 22, int(nan_payload.sum()))).astype(np.uint32) \
        | (rng.integers(0, 2, int(nan_payload.sum())).astype(np.uint32) << 31)
    return bits.view(np.float32)


def float_ops(n: int, wg: int = 64, seed: int = 0) -> Launch:
    """Each work-item applies every binary32 and integer operation of the
    machine to its pair (x[i], y[i]) and stores the 64-bit results in a row
    of len(FLOAT_OPS) words.  The expected rows come from the oracle."""
    K = len(FLOAT_OPS)
    A = Asm("float_ops")
    A.builtin("global_id", 4); A.icmp("ult", 5, 4, 3); A.br(5, "body", "end")
    A.label("body")
    A.gep(6, 0, 4, 4); A.load(7, 6, "u32"); A.gep(6, 1, 4, 4); A.load(8, 6, "u32")
    A.load(9, 6, "i32")                          # y as a signed integer
    A.mul(10, 4, I(8 * K)); A.gep(11, 2, 10, 1)  # row address
    r = 12
    ops = [lambda d: A.fadd(d, 7, 8), lambda d: A.fsub(d, 7, 8), lambda d: A.fmul(d, 7, 8),
           lambda d: A.fdiv(d, 7, 8), lambda d: A.fma(d, 7, 8, 7), lambda d: A.fsqrt(d, 7),
           lambda d: A.fmin(d, 7, 8), lambda d: A.fmax(d, 7, 8), lambda d: A.sitofp(d, 8),
           lambda d: A.fptosi(d, 7), lambda d: A.fcmp("olt", d, 7, 8),
           lambda d: A.fcmp("une", d, 7, 8)]
    for emit in ops:
        emit(r)
        A.store(11, r, size=8)
        A.gep(11, 11, offset=8)
    # integers: x widened with its sign, then shifted into the 64-bit range
    A.sext(20, 7); A.shl(21, 20, I(31)); A.or_(21, 21, 8)
    for emit in [lambda d: A.sdiv(d, 21, 9), lambda d: A.srem(d, 21, 9), lambda d: A.udiv(d, 21, 8),
                 lambda d: A.urem(d, 21, 8), lambda d: A.ashr(d, 21, 8), lambda d: A.shl(d, 21, 8),
                 lambda d: A.sext(d, 21), lambda d: A.zext(d, 21),
                 lambda d: A.select(d, 5, 21, 9)]:
        emit(r)
        A.store(11, r, size=8)
        A.gep(11, 11, offset=8)
    A.label("end"); A.ret()
    x = special_f32(n, seed)
    y = special_f32(n, seed + 1)
    out = np.zeros(n * K, dtype=np.uint64)
    g = -(-n // wg) * wg
    return Launch(A.finish(), (g,), (wg,), [Global(x), Global(y), Global(out), Scalar(n)],
                  names={"out": 2})
