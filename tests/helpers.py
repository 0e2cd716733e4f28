"""Small trace builders shared by the tests (input construction only)."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

OPDT = np.dtype([("op_class", "<u2"), ("simd_width", "u1"), ("kind", "u1")])
COMPUTE, LOAD, STORE, ATOMIC, BRANCH, BARRIER, OTHER = range(7)


def table(entries: Sequence[tuple]) -> np.ndarray:
    t = np.zeros(len(entries), dtype=OPDT)
    for i, e in enumerate(entries):
        t[i] = e
    return t


# a default table: id 0..3 compute (classes 0..3, width 1), 4 load, 5 store,
# 6 cond branch, 7 barrier, 8 ret, 9 atomic read-modify-write
DEFAULT_TABLE = table([(0, 1, COMPUTE), (1, 1, COMPUTE), (2, 1, COMPUTE), (3, 1, COMPUTE),
                       (4, 1, LOAD), (5, 1, STORE), (6, 1, BRANCH), (7, 1, BARRIER),
                       (8, 1, OTHER), (9, 1, ATOMIC)])
ID_LOAD, ID_STORE, ID_BRANCH, ID_BARRIER, ID_RET, ID_ATOMIC = 4, 5, 6, 7, 8, 9


@dataclass
class Trace:
    opcode: np.ndarray
    wi_offsets: np.ndarray
    addr: np.ndarray
    mem_kind: np.ndarray
    br_site: np.ndarray
    br_taken: np.ndarray
    n_sites: int = 1
    history_len: int = 16
    table: np.ndarray = field(default_factory=lambda: DEFAULT_TABLE.copy())


def mk(opcode=(), wi_lengths: Optional[Sequence[int]] = None, addr=(), mem_kind=None,
       br_site=(), br_taken=(), n_sites: int = 1, m: int = 16, tab=None) -> Trace:
    op = np.asarray(opcode, dtype=np.uint16)
    if wi_lengths is None:
        wi_lengths = [op.size]
    off = np.zeros(len(wi_lengths) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(np.asarray(wi_lengths, dtype=np.uint64))
    assert int(off[-1]) == op.size
    a = np.asarray(addr, dtype=np.uint64)
    k = np.zeros(a.size, dtype=np.uint8) if mem_kind is None else np.asarray(mem_kind, dtype=np.uint8)
    return Trace(op, off, a, k, np.asarray(br_site, dtype=np.uint32),
                 np.asarray(br_taken, dtype=np.uint8), n_sites=max(1, n_sites), history_len=m,
                 table=DEFAULT_TABLE.copy() if tab is None else tab)


def mem_trace(addr, kinds=None) -> Trace:
    """A trace whose only events are loads/stores of the given addresses."""
    a = np.asarray(addr, dtype=np.uint64)
    k = np.zeros(a.size, dtype=np.uint8) if kinds is None else np.asarray(kinds, dtype=np.uint8)
    op = np.where(k & 1, ID_STORE, ID_LOAD).astype(np.uint16)
    return mk(op, [op.size], a, k)


def branch_trace(sites, outcomes, n_sites: int, m: int) -> Trace:
    s = np.asarray(sites, dtype=np.uint32)
    op = np.full(s.size, ID_BRANCH, dtype=np.uint16)
    return mk(op, [op.size], br_site=s, br_taken=outcomes, n_sites=n_sites, m=m)


def random_trace(rng: np.random.Generator, n_wi: int, max_len: int, n_sites: int, m: int,
                 addr_bits: int = 12, p_local: float = 0.3) -> Trace:
    """Random small trace with consistent kinds (for brute-force checks).
    Atomic read-modify-writes issue a read and then a write of one address."""
    lens = rng.integers(0, max_len + 1, size=n_wi)
    n = int(lens.sum())
    ids = rng.integers(0, 10, size=n).astype(np.uint16)
    mem_ids = ids[np.isin(ids, [ID_LOAD, ID_STORE, ID_ATOMIC])]
    per = np.where(mem_ids == ID_ATOMIC, 2, 1)
    inst_addr = rng.integers(0, 1 << addr_bits, size=mem_ids.size, dtype=np.uint64)
    inst_local = (rng.random(mem_ids.size) < p_local).astype(np.uint8) << 1
    addr = np.repeat(inst_addr, per)
    kinds = np.repeat(inst_local, per)
    # write bit: stores, and the second event of each atomic
    first = np.concatenate([[0], np.cumsum(per)[:-1]]).astype(np.int64)
    w = np.zeros(addr.size, dtype=np.uint8)
    w[first[mem_ids == ID_STORE]] = 1
    w[first[mem_ids == ID_ATOMIC] + 1] = 1
    kinds = kinds | w
    nb = int((ids == ID_BRANCH).sum())
    sites = rng.integers(0, n_sites, size=nb).astype(np.uint32)
    taken = (rng.random(nb) < rng.random()).astype(np.uint8)
    return mk(ids, list(lens), addr, kinds, sites, taken, n_sites=n_sites, m=m)


def atomic_trace(addr, local=None) -> Trace:
    """One atomic read-modify-write per address: a read, then a write event."""
    a = np.asarray(addr, dtype=np.uint64)
    sp = np.zeros(a.size, dtype=np.uint8) if local is None else \
        (np.asarray(local, dtype=np.uint8) & 1) << 1
    ev = np.repeat(a, 2)
    kinds = np.repeat(sp, 2) | np.tile(np.array([0, 1], dtype=np.uint8), a.size)
    op = np.full(a.size, ID_ATOMIC, dtype=np.uint16)
    return mk(op, [op.size], ev, kinds)
