"""One persistent launch over many instances and uneven pools, checked against
single-pool launches and the oracle; graph replays checked after the node
buffers change between replays."""
import sys

import numpy as np
import pytest
import torch

from paper_1206_4973_amd import inputs as I

pytestmark = pytest.mark.gpu


def host_threads() -> int:
    """Host threads for the oracle (the CPU share of one GPU, at most 16)."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_4973_amd import fsp as F
    F.lib()
    return F


def mixed_batch(F, count_fn, seed0, shapes):
    items, host = [], []
    for i, (n, m) in enumerate(shapes):
        p = I.instance(n, m, seed0 + i)
        cnt = count_fn(i)
        pool = I.random_pool(n, cnt, 1, n - 1 if n > 1 else 1, seed0 + 500000 + i)
        inst = F.Instance(p)
        items.append((inst, torch.from_numpy(pool).cuda(), None))
        host.append((p, pool))
    return items, host


SHAPES = [(20, 5), (20, 10), (20, 20), (50, 5), (50, 10), (50, 20), (100, 5), (100, 10),
          (100, 20), (20, 7), (33, 20), (9, 5)]


def test_mixed_batch_matches_oracle_and_single_launches(fsp, orc):
    rng = np.random.default_rng(5)
    counts = [int(c) for c in rng.integers(1, 2500, size=len(SHAPES))]
    items, host = mixed_batch(fsp, lambda i: counts[i], 3100, SHAPES)
    b = fsp.Batch(items)
    info = b.info()
    say("batch info", info)
    assert info["kernel_segments"] == len(SHAPES) - 1 and info["fallback_segments"] == 1
    outs = b.launch()
    torch.cuda.synchronize()
    for (inst, nodes, _), out, (p, pool) in zip(items, outs, host):
        single = inst.bound_pool(nodes)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, single.cpu().numpy())
        assert np.array_equal(got, orc.bound_pool(p, pool, nthreads=8))
    b.close()


def test_forms_in_one_launch(fsp, orc):
    """Packed, 32-bit, 64-bit-register, bytes and job-mask segments in one
    launch (the same 20-job shape both packed and, with large times, 32-bit;
    a 200-job instance loaded for the job-mask walk keeps it; with job_masks
    the 100-job segment takes them too), with ragged tails of both tile
    sizes: every node equals the oracle, and the batch reports the form each
    segment took."""
    rng = np.random.default_rng(11)
    big = rng.integers(1500, 3000, size=(20, 10)).astype(np.int32)  # total > 32767
    cases = [(I.instance(20, 10, 3501), 1537), (big, 999), (I.instance(20, 20, 3502), 513),
             (I.instance(50, 10, 3503), 700), (I.instance(100, 5, 3504), 900),
             (I.instance(20, 5, 3505), 511), (I.instance(200, 10, 3506), 650)]
    items, host = [], []
    for i, (p, cnt) in enumerate(cases):
        n = p.shape[0]
        pool = I.random_pool(n, cnt, 0, n, 3600 + i)
        inst = fsp.Instance(p, job_masks=(i == 6))
        items.append((inst, torch.from_numpy(pool).cuda(), None))
        host.append((p, pool))
    b = fsp.Batch(items)
    paths, bpc = b.paths()
    say("paths", paths, "blocks per CU", bpc)
    assert paths == ["packed", "register", "packed", "register64", "bytes", "packed", "masks"]
    outs = b.launch()
    torch.cuda.synchronize()
    for out, (p, pool) in zip(outs, host):
        assert np.array_equal(out.cpu().numpy(), orc.bound_pool(p, pool, nthreads=8))
    b.close()
    bb = fsp.Batch(items, job_masks=True)
    assert bb.paths()[0] == ["packed", "register", "packed", "register64", "masks", "packed",
                             "masks"]
    outs = bb.launch()
    torch.cuda.synchronize()
    for out, (p, pool) in zip(outs, host):
        assert np.array_equal(out.cpu().numpy(), orc.bound_pool(p, pool, nthreads=8))
    bb.close()
    one = fsp.Batch(items, packed=False)
    assert one.paths()[0][0] == "register" and one.paths()[0][2] == "register"
    outs1 = one.launch()
    torch.cuda.synchronize()
    for o1, (p, pool) in zip(outs1, host):
        assert np.array_equal(o1.cpu().numpy(), orc.bound_pool(p, pool, nthreads=8))
    one.close()


def test_autotuned_batch_matches_oracle_and_caches(fsp, orc):
    """An autotuned batch (forms per shape and workgroups per CU timed on its
    own segments) bounds every node as the oracle does; a second batch of
    the same shapes takes the cached picks."""
    import time
    shapes = [(20, 10), (20, 20), (50, 20), (33, 5), (100, 10)]
    items, host = mixed_batch(fsp, lambda i: 3000 + 777 * i, 3700, shapes)
    t0 = time.perf_counter()
    b = fsp.Batch(items, autotune=True)
    t1 = time.perf_counter()
    paths, bpc = b.paths()
    say("autotuned paths", paths, "blocks per CU", bpc, f"planned in {t1 - t0:.3f} s")
    assert all(x is not None for x in paths) and bpc >= 1
    outs = b.replay()
    torch.cuda.synchronize()
    for out, (p, pool) in zip(outs, host):
        assert np.array_equal(out.cpu().numpy(), orc.bound_pool(p, pool, nthreads=8))
    b2 = fsp.Batch(items, autotune=True)
    assert b2.paths() == (paths, bpc)
    b.close()
    b2.close()


def test_one_shot_and_empty_segments(fsp, orc):
    items, host = mixed_batch(fsp, lambda i: [0, 700, 0][i], 3200, [(20, 20), (50, 10), (9, 5)])
    outs = fsp.bound_batch(items)
    assert outs[0].numel() == 0 and outs[2].numel() == 0
    assert np.array_equal(outs[1].cpu().numpy(), orc.bound_pool(*host[1], nthreads=8))


def test_graph_replay_sees_new_node_contents(fsp, orc):
    shapes = [(20, 20), (50, 10), (100, 5), (20, 7)]
    items, host = mixed_batch(fsp, lambda i: 900 + 300 * i, 3300, shapes)
    b = fsp.Batch(items)
    for rep in range(4):
        if rep:
            # eager work between replays: rewrite every pool in place
            for i, (inst, nodes, _) in enumerate(items):
                n = shapes[i][0]
                pool = I.random_pool(n, nodes.shape[0], 0, n, 3400 + 10 * rep + i)
                nodes.copy_(torch.from_numpy(pool))
                host[i] = (host[i][0], pool)
            torch.cuda.synchronize()
        outs = b.replay()
        torch.cuda.synchronize()
        for out, (p, pool) in zip(outs, host):
            assert np.array_equal(out.cpu().numpy(), orc.bound_pool(p, pool, nthreads=8)), rep
    b.close()


def test_batching_config_64_instances(fsp, orc):
    """64 instances, n in {20,50,100} x m in {5,10,20}, pools of 2^e nodes with e
    uniform in 10..18 (about 3.1 M nodes): every node of every segment equals
    the oracle, and every segment equals its single-pool launch."""
    shapes = [(n, m) for n in (20, 50, 100) for m in (5, 10, 20)]
    rng = np.random.default_rng(3000)
    exps = [int(e) for e in rng.integers(10, 19, size=64)]
    items, host = [], []
    say("generating 64 pools")
    for i in range(64):
        n, m = shapes[i % 9]
        p = I.instance(n, m, 3000 + i)
        pool = I.random_pool(n, 1 << exps[i], 1, n - 1, 3000 + 500000 + i)
        items.append((fsp.Instance(p), torch.from_numpy(pool).cuda(), None))
        host.append((p, pool))
    b = fsp.Batch(items)
    say("batch info", b.info(), "nodes", sum(1 << e for e in exps))
    outs = b.replay()
    torch.cuda.synchronize()
    for i, ((inst, nodes, _), out, (p, pool)) in enumerate(zip(items, outs, host)):
        got = out.cpu().numpy()
        ref = inst.bound_pool(nodes)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), i
        want = orc.bound_pool(p, pool, nthreads=host_threads())
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (i, bad[:10], got[bad[:10]], want[bad[:10]])
        if i % 8 == 7:
            say(f"  segments 0..{i} equal the oracle")
    b.close()
