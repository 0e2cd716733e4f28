"""The oracle's trace producer pinned against what the paper and the kernels
fix, independently of its own code: a hand-derived trace of a tiny kernel
(tests/golden/producer_tiny.json), kernel outputs equal to numpy / zlib /
a Python dynamic programme, closed-form event counts, the paper's schedule
order of branch events, binary32 results equal to numpy's, and the failing
cases (CPU only)."""
import json
import os

import numpy as np
import pytest

import oracle
from tracegen import kernels as K

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "producer_tiny.json")
T = 1 << K.ADDR_TAG_SHIFT


def tiny_program():
    A = K.Asm("tiny")
    A.builtin("local_id", 2)
    A.builtin("global_id", 3)
    A.gep(4, 0, 3, 4)
    A.load(5, 4, "u32")
    A.gep(6, 1, 2, 4)
    A.store(6, 5)
    A.barrier()
    A.icmp("eq", 7, 2, K.I(0))
    A.br(7, "take", "end")
    A.label("take")
    A.gep(8, 1, offset=4)
    A.load(9, 8, "u32")
    A.atomic("add", 10, 4, 9)
    A.label("end")
    A.ret()
    return A.finish()


def bits(a):
    return a.view(np.uint32) if a.dtype == np.float32 else a


def test_tiny_kernel_matches_the_hand_derived_trace():
    g = json.load(open(GOLDEN))
    prog = tiny_program()
    buf = np.array([10, 20, 30, 40], dtype=np.uint32)
    tr = oracle.produce(prog, (4,), (2,), [K.Global(buf), K.Local(8)])
    names = [prog.id_names[i] for i in tr.opcode]
    want = [n for wi in g["opcode_names"] for n in wi]
    assert names == want
    assert tr.wi_offsets.tolist() == g["wi_offsets"]
    ev = []
    for a, k, w in zip(tr.addr.tolist(), tr.mem_kind.tolist(), tr.mem_wi.tolist()):
        space = "local" if k & 2 else "global"
        base = "L" if k & 2 else "T"
        off = a if k & 2 else a - T
        ev.append([f"{base}+{off}", "write" if k & 1 else "read", space, w])
    assert ev == g["memory_events_in_execution_order"]
    assert [[s, t] for s, t in zip(tr.br_site.tolist(), tr.br_taken.tolist())] == g["branches"]
    assert buf.tolist() == g["buffer_after"]
    m = oracle.characterize(tr)
    gm = g["metrics"]
    assert m["total_instructions"] == gm["total_instructions"]
    assert m["work_items"] == gm["work_items"]
    assert m["barriers_hit"] == gm["barriers_hit"]
    assert m["itb_count"] == len(gm["itb_segments"]) and m["itb_sum"] == sum(gm["itb_segments"])
    assert (m["itb_min"], m["itb_max"]) == (min(gm["itb_segments"]), max(gm["itb_segments"]))
    assert (m["ipt_min"], m["ipt_max"]) == (min(gm["ipt"]), max(gm["ipt"]))
    assert m["space"][0]["footprint"] == gm["global_footprint"]
    assert m["space"][1]["footprint"] == gm["local_footprint"]
    # an atomic is one instruction with a read and a write event
    assert oracle.consistent(tr)


@pytest.mark.parametrize("launch", K.suite(), ids=lambda L: L.program.name)
def test_kernel_outputs_equal_independent_references(launch):
    args = launch.fresh_args()
    tr = oracle.produce(launch.program, launch.global_size, launch.local_size, args)
    for name, idx in launch.names.items():
        assert np.array_equal(bits(args[idx].array), bits(launch.expected[name])), name
    assert oracle.consistent(tr)
    assert int(tr.wi_offsets[-1]) == tr.opcode.size


def test_vector_add_closed_form_counts():
    n, wg = 1000, 256
    L = K.vector_add(n, wg=wg)
    tr = oracle.produce(L.program, L.global_size, L.local_size, L.fresh_args())
    ipt = np.diff(tr.wi_offsets.astype(np.int64))
    # in range: gid icmp br gep load gep load fadd gep store ret; else gid icmp br ret
    assert (ipt[:n] == 11).all() and (ipt[n:] == 4).all()
    assert tr.addr.size == 3 * n and tr.br_site.size == L.global_size[0]
    assert (tr.br_taken[:n] == 1).all() and (tr.br_taken[n:] == 0).all()
    m = oracle.characterize(tr)
    g = m["space"][0]
    assert g["footprint"] == 3 * n and g["unique_reads"] == 2 * n and g["unique_writes"] == n
    assert m["barriers_hit"] == 0 and m["itb_count"] == L.global_size[0]


def test_vector_add4_simd_width():
    L = K.vector_add4(100, wg=64)
    tr = oracle.produce(L.program, L.global_size, L.local_size, L.fresh_args())
    m = oracle.characterize(tr)
    # per in-range work-item: two 4-wide loads and one 4-wide fadd among 11 instructions
    assert m["simd_max"] == 4
    assert m["simd_sum"] == 100 * (8 + 3 * 4) + (128 - 100) * 4


def test_reduction_branch_stream_follows_the_schedule():
    """Inside a work-group, each work-item runs to the barrier before the next
    one starts, so the branch stream is ordered by barrier interval, then by
    local id (Implementation section)."""
    wg, n = 8, 16
    L = K.reduce_local(n, wg=wg)
    tr = oracle.produce(L.program, L.global_size, L.local_size, L.fresh_args())
    want = []
    for g in range(n // wg):
        want += [(0, 1)] * wg                   # interval 0: every gid < n
        s = wg // 2
        while s > 0:                            # one interval per tree level
            for lid in range(wg):
                want += [(1, 1), (2, int(lid < s))]
            s //= 2
        for lid in range(wg):                   # last interval: loop exit, writer
            want += [(1, 0), (3, int(lid == 0))]
    assert list(zip(tr.br_site.tolist(), tr.br_taken.tolist())) == want
    m = oracle.characterize(tr)
    levels = int(np.log2(wg))
    assert m["barriers_hit"] == n * (1 + levels)
    assert m["itb_count"] == n * (2 + levels)


def test_crc32_branch_counts():
    n_wi, words = 64, 3
    L = K.crc32(n_wi, words)
    tr = oracle.produce(L.program, L.global_size, L.local_size, L.fresh_args())
    # per word: the word-loop test, then per bit the parity and the bit-loop test; one final exit
    assert tr.br_site.size == n_wi * (words * (1 + 2 * 32) + 1)
    per_site = np.bincount(tr.br_site, minlength=3)
    assert per_site.tolist() == [n_wi * (words + 1), n_wi * words * 32, n_wi * words * 32]


def test_histogram_atomics_are_read_write_pairs():
    n, bins = 5000, 37
    L = K.histogram(n, bins, n_wi=512, wg=128)
    tr = oracle.produce(L.program, L.global_size, L.local_size, L.fresh_args())
    assert tr.addr.size == 3 * n
    m = oracle.characterize(tr)
    g = m["space"][0]
    assert g["total_reads"] == 2 * n and g["total_writes"] == n
    assert g["unique_writes"] == np.unique(L.args[0].array % bins).size


def test_binary32_operations_equal_numpy():
    L = K.float_ops(400, seed=3)
    args = L.fresh_args()
    oracle.produce(L.program, L.global_size, L.local_size, args)
    out = args[2].array.reshape(-1, len(K.FLOAT_OPS))
    x, y = args[0].array, args[1].array

    def canon(v):
        b = v.astype(np.float32).view(np.uint32).astype(np.uint64)
        b[np.isnan(v)] = 0x7FC00000
        return b

    with np.errstate(all="ignore"):
        ref = {"fadd": x + y, "fsub": x - y, "fmul": x * y, "fdiv": x / y, "fsqrt": np.sqrt(x)}
        for k, v in ref.items():
            assert np.array_equal(out[:, K.FLOAT_OPS.index(k)], canon(v)), k
        lt = out[:, K.FLOAT_OPS.index("fcmp_olt")]
        assert np.array_equal(lt, (x < y).astype(np.uint64))
        une = out[:, K.FLOAT_OPS.index("fcmp_une")]
        assert np.array_equal(une, (~(x == y)).astype(np.uint64))
        yi = y.view(np.int32).astype(np.float32)
        assert np.array_equal(out[:, K.FLOAT_OPS.index("sitofp")], canon(yi))
    fmin = out[:, K.FLOAT_OPS.index("fmin")].astype(np.uint32).view(np.float32)
    # numpy's fmin ignores NaNs like the machine does; signed zeros aside
    ref_min = np.fmin(x, y)
    same = ~((x == 0) & (y == 0))
    assert np.array_equal(np.isnan(fmin), np.isnan(ref_min))
    ok = same & ~np.isnan(ref_min)
    assert np.array_equal(fmin[ok], ref_min[ok])


def _one_wi(prog_fn, args, global_size=(1,), local_size=(1,), max_steps=0):
    A = K.Asm("probe")
    prog_fn(A)
    return oracle.produce(A.finish(), global_size, local_size, args, max_steps=max_steps)


def test_failing_kernels():
    buf = np.zeros(4, dtype=np.uint32)

    def oob(A):
        A.gep(1, 0, offset=16); A.load(2, 1, "u32"); A.ret()

    def misaligned(A):
        A.gep(1, 0, offset=2); A.load(2, 1, "u32"); A.ret()

    def spin(A):
        A.label("top"); A.mov(1, K.I(1)); A.br(1, "top", "out"); A.label("out"); A.ret()

    def off_end(A):
        A.mov(1, K.I(0))

    def lone_barrier(A):
        A.builtin("local_id", 1); A.icmp("eq", 2, 1, K.I(0)); A.br(2, "b", "e")
        A.label("b"); A.barrier(); A.label("e"); A.ret()

    cases = [(oob, 1, (1,), (1,)), (misaligned, 2, (1,), (1,)), (spin, 4, (1,), (1,)),
             (off_end, 16, (1,), (1,)), (lone_barrier, 8, (4,), (4,))]
    for fn, code, gs, ls in cases:
        with pytest.raises(oracle.ProduceError) as e:
            _one_wi(fn, [K.Global(buf.copy())], gs, ls, max_steps=1000)
        assert e.value.code == code, fn.__name__


def test_local_memory_is_per_work_group_and_zeroed():
    def prog(A):
        A.builtin("local_id", 2); A.gep(3, 1, 2, 4); A.load(4, 3, "u32"); A.add(4, 4, K.I(1))
        A.store(3, 4); A.builtin("global_id", 5); A.gep(6, 0, 5, 4); A.store(6, 4); A.ret()
    out = np.full(8, 99, dtype=np.uint32)
    tr = _one_wi(prog, [K.Global(out), K.Local(16)], (8,), (4,))
    assert out.tolist() == [1] * 8
    m = oracle.characterize(tr)
    assert m["space"][1]["footprint"] == 4 and m["space"][1]["total_accesses"] == 16
