"""Parity of the HIP pool-bounding kernel with the CPU oracle, through the C ABI.

Bounds are integers: every comparison is bit-exact.  Small pools span several
256-node tiles and a ragged tail and are compared element by element; so are
the benchmarked 20x20 pool of 2^22 nodes (on both the packed and the 32-bit
form) and a 50x20 pool of 2^20 nodes.  The 200x20 pool of 2^22 nodes is
compared on a random sample plus a property that holds for every node.
"""
import os
import sys

import numpy as np
import pytest
import torch

from paper_1206_4973_amd import inputs as I

pytestmark = pytest.mark.gpu

SHAPES = [(1, 2), (2, 2), (3, 3), (5, 4), (9, 5), (16, 7), (20, 5), (20, 10), (20, 20),
          (31, 20), (32, 20), (32, 3), (33, 20), (50, 5), (50, 10), (50, 20), (64, 13),
          (100, 5), (100, 10), (100, 20), (200, 20), (255, 20), (255, 2)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_4973_amd import fsp as F
    F.lib()  # raises if the library is missing
    return F


def gpu_bounds(F, inst, pool, stream=None):
    t = torch.from_numpy(np.ascontiguousarray(pool)).cuda()
    out = inst.bound_pool(t, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_tiny_config_pool(fsp, orc):
    """9 jobs x 5 machines, 4096 nodes of depth 0..8."""
    p = I.instance(9, 5, 1000)
    pool = I.random_pool(9, 4096, 0, 8, 1000 + 500000)
    say("tiny config: 4096 nodes, n=9 m=5")
    inst = fsp.Instance(p)
    got = gpu_bounds(fsp, inst, pool)
    want = orc.bound_pool(p, pool, nthreads=8)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,m", SHAPES, ids=[f"{n}x{m}" for n, m in SHAPES])
def test_shapes_bit_exact(fsp, orc, n, m):
    count = 1537 if n <= 100 else 600  # several tiles and a ragged tail
    p = I.instance(n, m, 7000 + 31 * n + m)
    pool = I.random_pool(n, count, 0, n, 8000 + 31 * n + m)
    say(f"shape n={n} m={m}: {count} nodes")
    want = orc.bound_pool(p, pool, nthreads=8)
    # above 64 jobs both walks: the bytes walk (default) and the job masks
    for masks in ((False, True) if n > 64 else (False,)):
        inst = fsp.Instance(p, job_masks=masks)
        got = gpu_bounds(fsp, inst, pool)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (inst.bound_path, bad[:10], got[bad[:10]], want[bad[:10]])


def test_zero_times_and_ties(fsp, orc):
    """Zero processing times and many equal keys (Johnson ties)."""
    rng = np.random.default_rng(3)
    for n, m in ((12, 6), (40, 9)):
        p = rng.integers(0, 3, size=(n, m)).astype(np.int32)
        pool = I.random_pool(n, 900, 0, n, 4 + n)
        inst = fsp.Instance(p)
        assert np.array_equal(gpu_bounds(fsp, inst, pool), orc.bound_pool(p, pool, 8))


def test_identical_jobs_and_two_machines(fsp, orc):
    c = np.array([5, 9, 2, 7], np.int32)
    p = np.tile(c, (10, 1))
    inst = fsp.Instance(p)
    root = I.records([[]], 10)
    assert gpu_bounds(fsp, inst, root)[0] == c.sum() + 9 * c.max()
    p2 = I.instance(7, 2, 99)
    pool = I.random_pool(7, 300, 0, 7, 98)
    inst2 = fsp.Instance(p2)
    got = gpu_bounds(fsp, inst2, pool)
    for i in range(0, 300, 11):
        d = int(pool[i, 0])
        assert got[i] == orc.best_completion(p2, pool[i, 1:1 + d].tolist())


def test_malformed_nodes(fsp, orc):
    for n in (20, 60):
        p = I.instance(n, 8, 5 + n)
        recs = I.random_pool(n, 300, 0, n, 6 + n)
        recs[3, 0] = n + 1                    # depth > n
        recs[7, 0] = max(2, recs[7, 0]); recs[7, 2] = recs[7, 1]   # duplicate
        recs[11, 0] = max(1, recs[11, 0]); recs[11, 1] = n         # id == n
        recs[13, 0] = max(1, recs[13, 0]); recs[13, 1] = 255       # id 255
        recs[17, 0] = 255                     # depth 255
        # the same faults on nodes 256 + i, which the packed path bounds in
        # the high halves of the lanes that hold nodes i
        recs[261, 0] = n + 1
        recs[265, 0] = max(2, recs[265, 0]); recs[265, 2] = recs[265, 1]
        recs[268, 0] = max(1, recs[268, 0]); recs[268, 1] = n
        recs[7 + 256, 0] = max(3, recs[7 + 256, 0]); recs[7 + 256, 3] = recs[7 + 256, 2]
        inst = fsp.Instance(p)
        got = gpu_bounds(fsp, inst, recs)
        want = orc.bound_pool(p, recs, 8)
        assert np.array_equal(got, want)
        for i in (3, 7, 11, 13, 17, 261, 263, 265, 268):
            assert got[i] == -1


def test_count_zero_and_argument_errors(fsp):
    inst = fsp.Instance(I.instance(8, 4, 1))
    empty = torch.zeros((0, 16), dtype=torch.uint8, device="cuda")
    out = inst.bound_pool(empty)
    assert out.numel() == 0
    short = torch.zeros((4, 8), dtype=torch.uint8, device="cuda")  # stride < n+1
    with pytest.raises(fsp.FspError):
        inst.bound_pool(short)


def test_unaligned_records(fsp, orc):
    """stride = n+1 (not a multiple of 16) and a base address offset by 1."""
    n, m = 20, 20
    p = I.instance(n, m, 2000)
    pool = I.random_pool(n, 1001, 1, 19, 2001, stride=n + 1)
    inst = fsp.Instance(p)
    flat = torch.zeros(1 + pool.size, dtype=torch.uint8, device="cuda")
    flat[1:] = torch.from_numpy(pool.reshape(-1)).cuda()
    view = flat[1:].view(1001, n + 1)
    out = inst.bound_pool(view)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), orc.bound_pool(p, pool, 8))


def test_non_default_stream_and_reuse(fsp, orc):
    n, m = 20, 10
    p = I.instance(n, m, 4000)
    inst = fsp.Instance(p)
    s = torch.cuda.Stream()
    pools = [I.random_pool(n, 5000 + 7 * i, 1, 19, 4100 + i) for i in range(3)]
    with torch.cuda.stream(s):
        outs = [inst.bound_pool(torch.from_numpy(q).cuda(), stream=s) for q in pools]
    s.synchronize()
    for q, o in zip(pools, outs):
        assert np.array_equal(o.cpu().numpy(), orc.bound_pool(p, q, 8))


def test_branching_shaped_pool(fsp, orc):
    n, m = 20, 20
    p = I.instance(n, m, 2000)
    pool = I.sibling_pool(n, 150, 0, n - 1, 2002)
    inst = fsp.Instance(p)
    assert np.array_equal(gpu_bounds(fsp, inst, pool), orc.bound_pool(p, pool, 8))


def host_threads() -> int:
    """Host threads for the oracle (the CPU share of one GPU, at most 16)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


_ORACLE_CACHE = {}


def oracle_full(orc, key, p, pool):
    """The oracle's bounds of a whole pool, computed once per module."""
    if key not in _ORACLE_CACHE:
        say(f"  oracle on all {len(pool)} nodes, {host_threads()} threads")
        _ORACLE_CACHE[key] = orc.bound_pool(p, pool, nthreads=host_threads())
    return _ORACLE_CACHE[key]


EVERY = [(20, 20, 2000, 22), (50, 20, 5000, 20)]


@pytest.mark.parametrize("n,m,seed,log2", EVERY, ids=["20x20_2p22", "50x20_2p20"])
def test_full_size_pool_every_node(fsp, orc, n, m, seed, log2):
    """The benchmarked 20x20 pool of 2^22 nodes (packed form, the launch the
    benchmark times) and a 50x20 pool of 2^20 nodes (64-bit register form):
    every node equals the oracle."""
    count = 1 << log2
    say(f"full size n={n} m={m}: generating {count} nodes")
    p = I.instance(n, m, seed)
    pool = I.random_pool(n, count, 1, n - 1, seed + 500000)
    inst = fsp.Instance(p)
    say(f"  bounding on the GPU ({inst.bound_path} form)")
    got = gpu_bounds(fsp, inst, pool)
    want = oracle_full(orc, (n, m, seed, log2), p, pool)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:10], got[bad[:10]], want[bad[:10]])


def test_full_size_pool_register_form(fsp, orc):
    """The same 2^22-node 20x20 pool on the one-node-per-lane 32-bit form
    (the packed form switched off at load): every node equals the oracle."""
    n, m, seed, log2 = 20, 20, 2000, 22
    p = I.instance(n, m, seed)
    pool = I.random_pool(n, 1 << log2, 1, n - 1, seed + 500000)
    inst = fsp.Instance(p, packed=False)
    assert inst.bound_path == "register"
    say("full size 20x20 on the register form")
    got = gpu_bounds(fsp, inst, pool)
    want = oracle_full(orc, (n, m, seed, log2), p, pool)
    assert np.array_equal(got, want)


def test_full_size_pool_sampled_200x20(fsp, orc):
    """200x20, 2^22 nodes (bytes walk, the default above 64 jobs): the oracle
    is too slow for every node, so 2048 random nodes and the last 37 are
    compared with it; every node bounds at least the root (the bound never
    decreases along a branch) and none is invalid.  The job-mask walk, an
    independent device path, gives the same bound on every node."""
    n, m, seed = 200, 20, 5001
    count = 1 << 22
    say(f"full size n={n} m={m}: generating {count} nodes")
    p = I.instance(n, m, seed)
    pool = I.random_pool(n, count, 1, n - 1, seed + 500000)
    inst = fsp.Instance(p)
    assert inst.bound_path == "bytes"
    say("  bounding on the GPU")
    got = gpu_bounds(fsp, inst, pool)
    masks = fsp.Instance(p, job_masks=True)
    assert masks.bound_path == "masks"
    say("  bounding on the GPU, job-mask walk")
    assert np.array_equal(gpu_bounds(fsp, masks, pool), got)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(count, size=2048, replace=False))
    idx = np.unique(np.concatenate([idx, np.arange(count - 37, count)]))
    say(f"  oracle on {len(idx)} nodes")
    want = orc.bound_pool(p, pool[idx], nthreads=host_threads())
    assert np.array_equal(got[idx], want)
    assert got.min() >= orc.lower_bound(p, [])


def _hip():
    """torch's HIP runtime (already loaded: same SONAME)."""
    import ctypes
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


RAGGED = [(20, 20, True), (20, 20, False), (50, 20, True), (100, 10, True)]


@pytest.mark.parametrize("n,m,packed", RAGGED,
                         ids=["20x20_packed", "20x20_register", "50x20", "100x10"])
def test_ragged_tail_in_exact_allocation(fsp, orc, n, m, packed):
    """A pool whose last tile is ragged (count not a multiple of the 512-node
    packed tile nor of the 256-node tile), in a buffer of exactly count *
    stride bytes from hipMalloc (where the stride allows it, a whole number
    of 4 KiB pages, so the pool ends where the mapped memory ends), bounded
    through the C ABI with raw device pointers: every node equals the
    oracle, and no lane past the end reads a record (a regression test of the
    packed form's record loads)."""
    import ctypes
    import math
    stride = ((n + 1) + 15) // 16 * 16
    whole_pages = 4096 // math.gcd(stride, 4096)  # smallest count filling whole pages
    count = 3 * 512 + (whole_pages if whole_pages < 256 else 77)
    assert count % 512 != 0 and count % 256 != 0
    p = I.instance(n, m, 6100 + n + m)
    pool = np.ascontiguousarray(I.random_pool(n, count, 0, n, 6200 + n + m))
    assert pool.shape == (count, stride)
    inst = fsp.Instance(p, packed=packed)
    say(f"exact allocation n={n} m={m} ({inst.bound_path}): {count} nodes, "
        f"{count * stride} bytes")
    hip = _hip()
    d_nodes, d_lb = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(d_nodes), count * stride) == 0
    assert hip.hipMalloc(ctypes.byref(d_lb), count * 4) == 0
    try:
        assert hip.hipMemcpy(d_nodes, pool.ctypes.data_as(ctypes.c_void_p),
                             count * stride, 1) == 0  # host to device
        desc = fsp._Nodes()
        desc.inst = inst.handle.value
        desc.data = d_nodes.value
        desc.stride = stride
        rc = fsp.lib().fsp_bound_pool(ctypes.byref(desc), count, d_lb, None)
        assert rc == 0, fsp.status_string(rc)
        assert hip.hipDeviceSynchronize() == 0
        got = np.empty(count, np.int32)
        assert hip.hipMemcpy(got.ctypes.data_as(ctypes.c_void_p), d_lb, count * 4, 2) == 0
    finally:
        hip.hipFree(d_nodes)
        hip.hipFree(d_lb)
    assert np.array_equal(got, orc.bound_pool(p, pool, nthreads=host_threads()))


@pytest.mark.parametrize("n,m,total,big", [(20, 20, 32767, 0), (20, 20, 32768, 0),
                                           (12, 6, 32767, 30000), (31, 20, 32767, 20000),
                                           (2, 2, 32767, 32767)])
def test_packed_path_limits(fsp, orc, n, m, total, big):
    """Instances whose total work sits at the limit of the two-nodes-per-lane
    16-bit path (<= 32767 takes it, 32768 does not), some with one processing
    time close to the largest 16-bit value: every bound must equal the
    oracle's."""
    rng = np.random.default_rng(total + n + big)
    p = rng.integers(0, 100, size=(n, m)).astype(np.int64)
    if big:
        p[0, m // 2] = big
    # put the difference on entries of other jobs (job totals stay <= 65535)
    diff = total - int(p.sum())
    j = 1 % n
    while diff != 0:
        k = int(rng.integers(0, m))
        step = max(-int(p[j, k]), min(diff, 32767 - int(p[j, k]), 65535 - int(p[j].sum())))
        p[j, k] += step
        diff -= step
        j = (j + 1) % n
    p = p.astype(np.int32)
    assert int(p.sum()) == total and p.max() <= 32767
    pool = I.random_pool(n, 2000, 0, n, 900000 + total + n)
    say(f"packed limit n={n} m={m} total={total} max p={int(p.max())}")
    inst = fsp.Instance(p)
    assert inst.bound_path == ("packed" if total <= 32767 else "register")
    got = gpu_bounds(fsp, inst, pool)
    want = orc.bound_pool(p, pool, nthreads=8)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,m", [(80, 4), (130, 7)])
def test_bytes_walk_records_at_the_instance_limits(fsp, orc, n, m):
    """The bytes walk packs each table position into one word, b - a in the
    low and lag + b in the high 16 bits, which the instance limits (times up
    to 32767, job totals up to 65535) keep in range.  Jobs that reach those
    limits, with b - a = +-32767 and lag + b = 65535 in some pairs, beside
    small ones: every bound equals the oracle's, on the bytes walk and on the
    job-mask walk."""
    rng = np.random.default_rng(n * 100 + m)
    p = rng.integers(1, 100, size=(n, m)).astype(np.int64)
    for j in range(8):
        row = np.zeros(m, np.int64)
        if j % 2 == 0:
            # pair (0, 3): a = 0, lag = 32767 + 1, b = 32767: b - a = 32767
            # and lag + b = 65535 (the job's total)
            row[1], row[2], row[3] = 32767, 1, 32767
        else:
            # pairs (0, l): a = 32767, b = 0: b - a = -32767
            row[0] = 32767
        p[j] = row
    p = p.astype(np.int32)
    assert p.max() <= 32767 and int(p.sum(axis=1).max()) <= 65535
    assert int(p.sum(axis=1).max()) == 65535
    assert int(p.sum()) < (1 << 22)
    pool = I.random_pool(n, 3000, 0, n, 910000 + n + m)
    want = orc.bound_pool(p, pool, nthreads=8)
    for masks in (False, True):
        inst = fsp.Instance(p, job_masks=masks)
        say(f"limits n={n} m={m} path {inst.bound_path}")
        assert inst.bound_path == ("masks" if masks else "bytes")
        got = gpu_bounds(fsp, inst, pool)
        inst.close()
        assert np.array_equal(got, want)


def test_concurrent_streams_with_job_mask_scratch(fsp, orc):
    """Instances above 64 jobs on the job-mask walk bound with per-wave mask
    scratch that the library keeps per stream: two streams bounding different
    pools at the same time, then a larger pool on the first stream (its
    workspace grows), must all match the oracle."""
    p = I.instance(100, 5, 7101)
    inst = fsp.Instance(p, job_masks=True)
    assert inst.bound_path == "masks"
    pools = [I.random_pool(100, c, 0, 100, 7200 + c) for c in (3000, 2500, 9000)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dev = [torch.from_numpy(np.ascontiguousarray(q)).cuda() for q in pools]
    torch.cuda.synchronize()
    say("two streams, 100x5, pools of 3000 and 2500 nodes, then 9000")
    out1 = inst.bound_pool(dev[0], stream=s1)
    out2 = inst.bound_pool(dev[1], stream=s2)
    out3 = inst.bound_pool(dev[2], stream=s1)
    torch.cuda.synchronize()
    for q, o in zip(pools, (out1, out2, out3)):
        assert np.array_equal(o.cpu().numpy(), orc.bound_pool(p, q, nthreads=8))



@pytest.mark.parametrize("n,m", [(9, 5), (20, 20), (31, 20), (32, 20), (20, 10), (50, 20),
                                 (64, 13), (100, 10), (255, 3)],
                         ids=lambda v: str(v))
def test_one_machine_bound_matches_oracle(fsp, orc, n, m):
    """fsp_bound_pool_one_machine in every walk form (packed, register,
    register64, masks) against the oracle's one-machine bound, bit for bit,
    and never above the pair bound."""
    count = 1537 if n <= 100 else 700
    p = I.instance(n, m, 8100 + 7 * n + m)
    pool = I.random_pool(n, count, 0, n, 8200 + 7 * n + m)
    say(f"one-machine bound n={n} m={m}: {count} nodes")
    inst = fsp.Instance(p)
    t = torch.from_numpy(np.ascontiguousarray(pool)).cuda()
    got = inst.bound_pool_one_machine(t)
    both = inst.bound_pool(t)
    torch.cuda.synchronize()
    got, both = got.cpu().numpy(), both.cpu().numpy()
    want = orc.bound_pool_one_machine(p, pool, nthreads=8)
    assert np.array_equal(got, want)
    assert np.all(got <= both)
