"""Host logic of the serving form (CPU only): the pool allocator and the
admission footprint."""

import math

import pytest

serve = pytest.importorskip("paper_2207_06374_amd.serve")


def test_allocator_first_fit_merge_and_peak():
    a = serve.OffsetAllocator(4096)
    x = a.alloc(1000)            # rounds to 1024
    y = a.alloc(1024)
    z = a.alloc(2048)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(1) is None and a.used == 4096 and a.peak == 4096
    a.release(y, 1024)
    assert a.alloc(2048) is None            # only 1024 free
    a.release(x, 1000)
    assert a.free == [(0, 2048)]            # merged with the neighbour
    assert a.alloc(2048) == 0
    a.release(0, 2048)
    a.release(z, 2048)
    assert a.free == [(0, 4096)] and a.used == 0


def test_allocator_never_exceeds_capacity():
    import random
    rnd = random.Random(0)
    a = serve.OffsetAllocator(1 << 20)
    live = []
    for _ in range(2000):
        if live and rnd.random() < 0.5:
            off, size = live.pop(rnd.randrange(len(live)))
            a.release(off, size)
        else:
            size = rnd.randrange(1, 1 << 16)
            off = a.alloc(size)
            if off is not None:
                for o, s in live:
                    assert off + serve.OffsetAllocator.round(size) <= o or o + serve.OffsetAllocator.round(s) <= off
                live.append((off, size))
        assert 0 <= a.used <= a.capacity and a.peak <= a.capacity


def test_welch_target():
    assert serve.welch_bound(16, 8) == math.sqrt(8 / (8 * 15))
    assert serve.welch_bound(4, 8) == 0.0
