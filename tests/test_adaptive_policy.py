"""Algorithm 1 (the paper's dynamic parameter tuning, Sec. III) as the
library implements it for FSP_POOL_ADAPTIVE: the pool size it sets batch by
batch for a given sequence of measured efficiencies.  The schedule is host
code (fsp_adaptive_schedule), so this runs on the CPU.

Expected sequences are written out from the algorithm's description: start
at threads-per-block x #compute units, double after every batch of
nb_iterations pools while the size stays within the device's resident-thread
maximum, then search around the best size -- the midpoints between the best
and the ends of [best/2, 2 best], two rounds with the interval narrowed
around the best after each -- and keep the best size from then on."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1206_4973_amd", "libfsp.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libfsp.so is not built (python -m paper_1206_4973_amd.build)")
    lib = ctypes.CDLL(LIB)
    i32, i64, P = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.fsp_adaptive_schedule.argtypes = [i32, i32, i64, i64, P, i32, P]
    lib.fsp_adaptive_schedule.restype = ctypes.c_int
    return lib


def schedule(L, eff, cus=256, max_threads=256 * 2048, max_pool=0, tpb=256):
    e = np.ascontiguousarray(eff, dtype=np.float64)
    out = np.zeros(len(e), dtype=np.int64)
    rc = L.fsp_adaptive_schedule(tpb, cus, max_threads, max_pool,
                                 e.ctypes.data_as(ctypes.c_void_p), len(e),
                                 out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    return [int(x) for x in out]


def eff_peaked_at(peak):
    """Efficiency as a function of the pool size, highest at `peak`."""
    return lambda size: 1e10 - abs(np.log2(size) - np.log2(peak)) * 1e8


def run(L, curve, batches, **kw):
    """Feed the efficiency of each size the schedule picks back into it."""
    effs, targets = [], []
    for _ in range(batches):
        t = schedule(L, effs + [0.0], **kw)[-1]
        targets.append(t)
        effs.append(curve(t))
    assert schedule(L, effs, **kw) == targets
    return targets


def test_doubling_then_search_then_freeze(L):
    # MI355X-like device: 256 compute units x 2048 resident threads = 524288
    got = run(L, eff_peaked_at(262144), 12)
    assert got == [65536, 131072, 262144, 524288,        # doubling from 256 x 256
                   196608, 393216,                       # midpoints of [131072, 524288]
                   229376, 327680,                       # narrowed to [196608, 393216]
                   262144, 262144, 262144, 262144]       # frozen at the best


def test_best_at_the_device_maximum(L):
    got = run(L, eff_peaked_at(1 << 30), 10)
    assert got[:4] == [65536, 131072, 262144, 524288]
    # midpoints around the best (524288) are clamped to the maximum
    assert got[4:8] == [393216, 524288, 458752, 524288]
    assert got[8:] == [524288, 524288]


def test_best_at_the_start(L):
    # smaller is better: each midpoint below the best becomes the new best
    got = run(L, eff_peaked_at(1), 10)
    assert got[:4] == [65536, 131072, 262144, 524288]
    assert got[4:6] == [49152,                  # (32768 + 65536) / 2: better
                        90112]                  # (49152 + 131072) / 2
    # narrowed: lo = (32768 + 49152) / 2, hi = (49152 + 131072) / 2
    assert got[6:8] == [45056,                  # (40960 + 49152) / 2: better
                        67584]                  # (45056 + 90112) / 2
    assert got[8:] == [45056, 45056]


def test_pool_cap_ends_the_doubling(L):
    # max_pool below the device maximum: doubling stops at 131072 (the next
    # size, 262144, exceeds 200000); sizes above the cap are clamped to it
    got = run(L, eff_peaked_at(1 << 30), 8, max_pool=200000)
    assert got == [65536, 131072,
                   98304, 196608,               # midpoints of [65536, 262144]; 196608 is better
                   163840, 200000,              # narrowed to [131072, 229376]; 212992
                                                # clamped to the cap, which is better
                   200000, 200000]              # frozen at the cap


def test_ties_keep_the_first_best(L):
    # equal efficiencies: "improved" means strictly better, so the first
    # size stays the best and the search centres on it
    got = schedule(L, [5.0] * 10)
    assert got == [65536, 131072, 262144, 524288,
                   49152, 98304,                # midpoints of [32768, 131072]
                   57344, 81920,                # narrowed to [49152, 98304]
                   65536, 65536]


def test_rejects_bad_arguments(L):
    out = np.zeros(2, np.int64)
    e = np.zeros(2)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.fsp_adaptive_schedule(0, 256, 1 << 19, 0, P(e), 2, P(out)) == -1
    assert L.fsp_adaptive_schedule(256, 0, 1 << 19, 0, P(e), 2, P(out)) == -1
    assert L.fsp_adaptive_schedule(256, 256, 1 << 19, 0, None, 2, P(out)) == -1
    assert L.fsp_adaptive_schedule(256, 256, 1 << 19, 0, P(e), -1, P(out)) == -1
