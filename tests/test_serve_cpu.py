"""CPU tests of the serving loop's host logic (allocator, footprints)."""
import pytest

from paper_1407_3383_amd import serve


class _FakeArena(serve.Arena):
    def __init__(self, budget):  # no device buffer
        self.budget = budget
        self.free = [(0, budget)]
        self.used = 0


def test_arena_first_fit_and_coalescing():
    a = _FakeArena(4096)
    o1 = a.alloc(100)
    o2 = a.alloc(1000)
    o3 = a.alloc(300)
    assert (o1, o2) == (0, 256) and o3 == 256 + 1024
    assert a.alloc(4096) is None
    a.release(o2, 1000)
    assert a.alloc(900) == 256              # reuses the hole
    a.release(256, 900)
    a.release(o1, 100)
    a.release(o3, 300)
    assert a.free == [(0, 4096)] and a.used == 0


def test_butterfly_count():
    assert serve.butterflies(4096, 4096) == 3 * 4096 * 13
    assert serve.butterflies(1, 1) == 0
    assert serve.butterflies(1 << 15, 1 << 15) == 3 * (1 << 15) * 16
