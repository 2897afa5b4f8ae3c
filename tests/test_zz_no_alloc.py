"""fsp_bound_pool_noalloc, the bounding entry point that allocates nothing,
through the C ABI: its bounds equal fsp_bound_pool's bit for bit on two calls
in a row (the second with a smaller pool, so a stale scratch would show), for
instances that need the fixed scratch (the job-mask walk, n > 64, loaded with
FSP_LOAD_JOB_MASKS) and for those that need none (every other walk); a pool
beyond the fixed scratch is refused before any device work."""
import sys

import numpy as np
import pytest
import torch

from paper_1206_4973_amd import inputs as I

pytestmark = pytest.mark.gpu

# (n, m, first pool, second pool, job-mask walk)
CASES = [(100, 20, 30001, 4099, True), (200, 10, 20480, 2561, True),
         (255, 5, 9000, 700, True), (80, 3, 70000, 513, True),
         (200, 10, 20480, 2561, False), (20, 20, 5000, 1537, False),
         (50, 10, 6000, 300, False)]


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


@pytest.mark.parametrize("n,m,first,second,masks", CASES,
                         ids=[f"{n}x{m}{'_masks' if k else ''}" for n, m, _, _, k in CASES])
def test_noalloc_equals_bound_pool_on_two_calls(fsp, orc, n, m, first, second, masks):
    p = I.instance(n, m, 9100 + n + m)
    inst = fsp.Instance(p, job_masks=masks)
    assert first <= inst.noalloc_max_count
    stream = torch.cuda.current_stream()
    for call, count in enumerate((first, second)):
        pool = I.random_pool(n, count, 0, n, 9200 + 7 * n + m + call)
        say(f"noalloc {n}x{m} call {call}: {count} nodes ({inst.bound_path})")
        nodes = torch.from_numpy(pool).cuda()
        want = torch.full((count,), -7, dtype=torch.int32, device="cuda")
        got = torch.full((count,), -7, dtype=torch.int32, device="cuda")
        inst.bound_pool(nodes, want, stream=stream)
        inst.bound_pool_noalloc(nodes, got, stream=stream)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        bad = np.nonzero(g != w)[0]
        assert bad.size == 0, (bad[:8], g[bad[:8]], w[bad[:8]])
        # and a sample against the oracle, the ragged tail included
        idx = np.unique(np.concatenate([np.arange(0, count, max(1, count // 300)),
                                        np.arange(max(0, count - 64), count)]))
        assert np.array_equal(g[idx], orc.bound_pool(p, pool[idx], nthreads=8))


def test_noalloc_refuses_a_pool_beyond_its_scratch(fsp):
    n, m = 255, 4
    inst = fsp.Instance(I.instance(n, m, 9300), job_masks=True)
    cap = inst.noalloc_max_count
    assert 0 < cap < 1 << 40
    count = cap + 1
    say(f"noalloc refusal: n={n}, {count} nodes > {cap}")
    nodes = torch.zeros((count, I.node_stride(n)), dtype=torch.uint8, device="cuda")
    out = torch.zeros(count, dtype=torch.int32, device="cuda")
    with pytest.raises(fsp.FspError) as e:
        inst.bound_pool_noalloc(nodes, out)
    assert e.value.rc == fsp.FSP_ESCRATCH
    torch.cuda.synchronize()
    assert int(out.abs().sum()) == 0  # nothing was queued
    small = fsp.Instance(I.instance(20, 5, 9301))
    assert small.noalloc_max_count == (1 << 63) - 1
    # the bytes walk (the default above 64 jobs) takes no scratch
    assert fsp.Instance(I.instance(n, m, 9300)).noalloc_max_count == (1 << 63) - 1
