"""The GPU trace producer against the oracle's (run with -m gpu): the same
kernel programs and inputs give identical opcode streams and work-item
offsets, identical memory events per work-item (their order across
work-items is free), identical branch streams in the paper's schedule
order, identical buffers afterwards, and metrics that agree with the
oracle's characterization of the oracle's trace."""
import numpy as np
import pytest
import torch

import oracle
from oracle.compare import compare
from tracegen import kernels as K

pytestmark = pytest.mark.gpu


def _gpu_args(launch):
    import paper_1805_04207_amd.aiwc as A
    args, dev = [], []
    for a in launch.args:
        if isinstance(a, K.Global):
            t = torch.from_numpy(a.array.copy().view(np.uint8)).to("cuda:0")
            dev.append(t)
            args.append((A.ARG_GLOBAL, t))
        elif isinstance(a, K.Local):
            dev.append(None)
            args.append((A.ARG_LOCAL, a.nbytes))
        else:
            dev.append(None)
            args.append((A.ARG_SCALAR, a.value))
    return args, dev


def run_both(launch, max_steps=0):
    from gpu_util import ctx
    c = ctx()
    p = launch.program
    prog = c.program(p.code, p.table, p.n_sites)
    args, dev = _gpu_args(launch)
    print(f"produce {p.name} global={launch.global_size} local={launch.local_size}", flush=True)
    produced = prog.produce(launch.global_size, launch.local_size, args, max_steps=max_steps)
    torch.cuda.synchronize()
    host_args = launch.fresh_args()
    want = oracle.produce(p, launch.global_size, launch.local_size, host_args, max_steps=max_steps)
    return c, prog, produced, dev, host_args, want


def check_arrays(got, want):
    assert np.array_equal(got["wi_offsets"], want.wi_offsets)
    assert np.array_equal(got["opcode"], want.opcode)
    # memory events: the GPU writes them work-item major; the oracle in
    # execution order with each event's work-item
    order = np.argsort(want.mem_wi, kind="stable")
    assert np.array_equal(got["addr"], want.addr[order])
    assert np.array_equal(got["mem_kind"], want.mem_kind[order])
    assert np.array_equal(got["br_site"], want.br_site)
    assert np.array_equal(got["br_taken"], want.br_taken)


@pytest.mark.parametrize("scale", [1, 3])
def test_suite_matches_the_oracle(scale):
    for launch in K.suite(scale=scale, seed=10 * scale):
        c, prog, produced, dev, host_args, want = run_both(launch)
        check_arrays(produced.to_host(), want)
        for i, t in enumerate(dev):
            if t is not None:
                assert np.array_equal(t.cpu().numpy(), host_args[i].array.view(np.uint8)), \
                    (launch.program.name, i)
        for name, idx in launch.names.items():
            got = dev[idx].cpu().numpy().view(launch.expected[name].dtype)
            assert np.array_equal(got.view(np.uint8), launch.expected[name].view(np.uint8)), name
        tr = produced.trace()
        got_m = c.characterize(tr).read()
        bad = compare(got_m, oracle.characterize(want))
        assert not bad, (launch.program.name, bad[:5])


def test_binary32_and_integer_semantics_bit_exact():
    launch = K.float_ops(2000, seed=5)
    c, prog, produced, dev, host_args, want = run_both(launch)
    got = dev[2].cpu().numpy().view(np.uint64).reshape(-1, len(K.FLOAT_OPS))
    exp = host_args[2].array.reshape(-1, len(K.FLOAT_OPS))
    for k, name in enumerate(K.FLOAT_OPS):
        bad = np.nonzero(got[:, k] != exp[:, k])[0]
        assert bad.size == 0, (name, [(hex(got[i, k]), hex(exp[i, k])) for i in bad[:4]])
    check_arrays(produced.to_host(), want)


def test_hot_histogram_and_wide_groups():
    for launch in (K.histogram(200000, 16, n_wi=8192, wg=1024, seed=3, zipf=1.5),
                   K.histogram_local(100000, 256, n_wi=4096, wg=512, seed=4),
                   K.reduce_local(70000, wg=1024, seed=5)):
        c, prog, produced, dev, host_args, want = run_both(launch)
        check_arrays(produced.to_host(), want)
        for name, idx in launch.names.items():
            got = dev[idx].cpu().numpy().view(launch.expected[name].dtype)
            assert np.array_equal(got, launch.expected[name]), name


def test_failing_kernels_leave_buffers_unchanged():
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()

    def build(fn):
        A = K.Asm("probe")
        fn(A)
        return A.finish()

    def oob(A):
        A.builtin("global_id", 1); A.gep(2, 0, 1, 4); A.store(2, K.I(7))
        A.gep(2, 0, offset=1 << 20); A.load(3, 2, "u32"); A.ret()

    def spin(A):
        A.builtin("global_id", 1); A.gep(2, 0, 1, 4); A.store(2, K.I(7))
        A.label("top"); A.mov(1, K.I(1)); A.br(1, "top", "out"); A.label("out"); A.ret()

    def lone_barrier(A):
        A.builtin("local_id", 1); A.icmp("eq", 2, 1, K.I(0)); A.br(2, "b", "e")
        A.label("b"); A.barrier(); A.label("e"); A.ret()

    def off_end(A):
        A.builtin("global_id", 1)

    for fn, word in ((oob, "left its buffer"), (spin, "max_steps"),
                     (lone_barrier, "barrier"), (off_end, "past the end")):
        p = build(fn)
        prog = c.program(p.code, p.table, p.n_sites)
        buf = torch.zeros(256, dtype=torch.int32, device="cuda:0")
        print(f"failing kernel {fn.__name__}", flush=True)
        with pytest.raises(aiwc.AiwcError) as e:
            prog.produce((256,), (64,), [(aiwc.aiwc.ARG_GLOBAL, buf)], max_steps=5000)
        assert e.value.status == aiwc.aiwc.AIWC_ERR_INVALID_ARG and word in str(e.value), str(e.value)
        assert int(buf.sum().item()) == 0, fn.__name__


def test_invalid_programs_are_rejected():
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    good = K.vector_add(10).program
    for field, value in (("op", 200), ("d", 63), ("id", 999), ("target2", 5000), ("width", 0)):
        code = good.code.copy()
        i = 8 if field == "d" else 2          # instruction 8 is a 1-wide gep; 2 is the branch
        if field == "d":
            code[i]["width"] = 4
        code[i][field] = value
        with pytest.raises(aiwc.AiwcError) as e:
            c.program(code, good.table, good.n_sites)
        assert e.value.status == aiwc.aiwc.AIWC_ERR_INVALID_ARG, field
    # a load whose opcode id claims the store kind
    code = good.code.copy()
    load_i = int(np.nonzero(code["op"] == K.LOAD)[0][0])
    store_i = int(np.nonzero(code["op"] == K.STORE)[0][0])
    code[load_i]["id"] = code[store_i]["id"]
    with pytest.raises(aiwc.AiwcError):
        c.program(code, good.table, good.n_sites)
