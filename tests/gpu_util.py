"""Helpers shared by the GPU tests: device setup and oracle comparisons."""
import sys

import numpy as np
import pytest


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_equal_u(actual: np.ndarray, expected: np.ndarray, what: str):
    actual = np.asarray(actual).astype(np.uint64)
    expected = np.asarray(expected).astype(np.uint64)
    assert actual.shape == expected.shape, (what, actual.shape, expected.shape)
    bad = np.nonzero(actual != expected)[0]
    assert bad.size == 0, "%s: %d mismatches, first at %d: got %d want %d" % (
        what, bad.size, bad[0], actual[bad[0]], expected[bad[0]])


def oracle_many(fn, args_list, workers: int = 0):
    """fn(*args) for every tuple of args_list on a pool of threads (the oracle's C
    routines release the GIL while they run), results in order."""
    import concurrent.futures as cf
    import os
    if workers <= 0:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda a: fn(*a), args_list))
