"""Host trace generator: determinism, internal consistency and marginals."""
import numpy as np

import tracegen as tg


def test_thread_count_does_not_change_bytes():
    spec = tg.config1()
    a = tg.generate_host(spec, threads=1)
    b = tg.generate_host(spec, threads=7)
    for f in ("opcode", "wi_offsets", "addr", "mem_kind", "br_site", "br_taken"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_kinds_match_streams_and_marginals():
    h = tg.generate_host(tg.config1())
    cnt = np.bincount(h.opcode, minlength=tg.N_OPCODE_IDS)
    assert cnt[tg.ID_LOAD] + cnt[tg.ID_STORE] == h.addr.size
    assert cnt[tg.ID_STORE] == int((h.mem_kind & 1).sum())
    assert cnt[tg.ID_BRANCH] == h.br_site.size
    assert cnt[tg.ID_RET] == 256 and int(h.wi_offsets[-1]) == h.opcode.size
    n = h.opcode.size - cnt[tg.ID_RET] - cnt[tg.ID_BARRIER]
    assert abs(h.addr.size / n - 0.30) < 0.01 and abs(h.br_site.size / n - 0.05) < 0.005
    assert h.addr.min() >= 1 << 28 and h.addr.max() < (1 << 28) + (1 << 19)
    assert (h.addr % 4 == 0).all() and h.br_site.max() < 16


def test_config2_family_small_has_both_spaces():
    spec = tg.config2(n_wi=512)
    h = tg.generate_host(spec)
    local = (h.mem_kind & 2) != 0
    assert 0.07 < local.mean() < 0.13
    assert h.addr[local].max() < 4 * (1 << 14)
    assert h.br_site.max() < 4096
