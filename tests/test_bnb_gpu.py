"""Device-resident branch-and-bound against the oracle, through the C ABI.

The optimum is unique (compared exactly); the schedule is not, so a returned
schedule is checked by recomputing its makespan.  With the initial UB set to
the optimum the set of bounded nodes no longer depends on the order of
exploration (every node whose bound is below the optimum is branched, every
child of a branched node is bounded), so the node counts must equal the
oracle's exactly under every pool policy.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1206_4973_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def check_schedule(orc, p, res):
    n = p.shape[0]
    assert sorted(res.perm.tolist()) == list(range(n))
    assert orc.makespan(p, res.perm) == res.makespan


def test_tiny_config_against_all_schedules(fsp, orc):
    """9 jobs x 5 machines: optimum = minimum over all 9! schedules."""
    p = I.instance(9, 5, 1000)
    opt, _ = orc.brute_force(p)
    inst = fsp.Instance(p)
    for kind, kw in (("adaptive", {}), ("fixed", {"fixed_pool": 1}),
                     ("fixed", {"fixed_pool": 64}), ("fixed", {"fixed_pool": 5000})):
        say(f"9x5 {kind} {kw}")
        res = fsp.branch_and_bound(inst, kind, **kw)
        assert res.status == 0 and res.makespan == opt
        check_schedule(orc, p, res)


@pytest.mark.parametrize("rule", ["ge", "gt"])
def test_random_small_instances(fsp, orc, rule):
    rng = np.random.default_rng(31 if rule == "ge" else 32)
    for t in range(12):
        n, m = int(rng.integers(2, 9)), int(rng.integers(2, 8))
        p = rng.integers(1, 99, size=(n, m)).astype(np.int32)
        opt, _ = orc.brute_force(p)
        inst = fsp.Instance(p)
        pool = int(rng.choice([1, 3, 50, 1000]))
        res = fsp.branch_and_bound(inst, "fixed", fixed_pool=pool, prune_rule=rule)
        assert res.makespan == opt, (n, m, pool)
        check_schedule(orc, p, res)


def test_neh_matches_oracle(fsp, orc):
    for n, m, seed in ((9, 5, 1000), (20, 20, 2000), (20, 10, 4000), (50, 20, 5000)):
        p = I.instance(n, m, seed)
        c, perm = fsp.neh(fsp.Instance(p))
        oc, operm = orc.neh(p)
        assert c == oc and np.array_equal(perm, operm)


SCREENED = [(12, 6, 61), (12, 8, 62), (13, 5, 63), (14, 7, 65), (15, 6, 67), (14, 8, 69),
            (15, 10, 70), (20, 10, 4046), (20, 10, 4052), (20, 10, 4056)]


@pytest.mark.parametrize("n,m,seed", SCREENED, ids=[f"{n}x{m}" for n, m, _ in SCREENED])
def test_optimum_matches_oracle_dfs(fsp, orc, n, m, seed):
    p = I.instance(n, m, seed)
    oc, _, ost = orc.bnb(p)
    assert ost.complete == 1
    inst = fsp.Instance(p)
    say(f"{n}x{m}: oracle {oc} after {ost.nodes_bounded} nodes")
    res = fsp.branch_and_bound(inst, "adaptive")
    assert res.status == 0 and res.makespan == oc
    assert res.root_lb == ost.root_lb
    check_schedule(orc, p, res)


@pytest.mark.parametrize("rule", ["ge", "gt"])
@pytest.mark.parametrize("n,m,seed", [(9, 5, 1000), (11, 7, 71), (12, 6, 61)])
def test_critical_tree_counts_equal_oracle(fsp, orc, n, m, seed, rule):
    p = I.instance(n, m, seed)
    opt, _, _ = orc.bnb(p)
    oc, _, ost = orc.bnb(p, opt, 0 if rule == "ge" else 1)
    assert oc == opt and ost.complete == 1
    inst = fsp.Instance(p)
    model = fsp.Model(2 + 2 * min(m, 15), 2, seed=seed)
    for kind, kw in (("fixed", {"fixed_pool": 1}), ("fixed", {"fixed_pool": 37}),
                     ("fixed", {"fixed_pool": 100000}), ("adaptive", {}),
                     ("autotuned", {"fixed_pool": 64}), ("learned", {"fixed_pool": 5, "model": model}),
                     ("learned", {"fixed_pool": 3000, "model": model}),
                     # the one-machine pre-filter skips pair walks, never an elimination
                     ("fixed", {"fixed_pool": 37, "prefilter": True}),
                     ("adaptive", {"prefilter": True}),
                     ("autotuned", {"fixed_pool": 64, "prefilter": True}),
                     ("learned", {"fixed_pool": 3000, "model": model, "prefilter": True}),
                     # hybrid: host threads search subtrees handed over by the device
                     ("fixed", {"fixed_pool": 37, "host_threads": 4}),
                     ("adaptive", {"host_threads": 3}),
                     ("autotuned", {"fixed_pool": 64, "host_threads": 4}),
                     ("learned", {"fixed_pool": 3000, "model": model, "host_threads": 2})):
        res = fsp.branch_and_bound(inst, kind, ub=opt, prune_rule=rule, **kw)
        say(f"{n}x{m} {rule} {kind} {kw}: {res.nodes_bounded} vs {ost.nodes_bounded}")
        assert res.makespan == opt and res.found == 0 and res.status == 0
        assert res.nodes_bounded == ost.nodes_bounded
        assert res.nodes_branched == ost.nodes_branched
        assert res.leaves == ost.leaves
        assert res.nodes_pruned == ost.nodes_pruned


def test_time_limit_returns_a_valid_schedule(fsp, orc):
    p = I.instance(20, 10, 4000)
    inst = fsp.Instance(p)
    neh_c, _ = orc.neh(p)
    res = fsp.branch_and_bound(inst, "adaptive", time_limit=1e-6)
    assert res.status == 1
    assert res.makespan <= neh_c
    check_schedule(orc, p, res)


def test_repeat_runs_give_the_same_optimum(fsp, orc):
    p = I.instance(12, 8, 62)
    inst = fsp.Instance(p)
    vals = {fsp.branch_and_bound(inst, "fixed", fixed_pool=200).makespan for _ in range(6)}
    assert len(vals) == 1


def test_policy_errors(fsp):
    inst = fsp.Instance(I.instance(8, 4, 3))
    with pytest.raises(fsp.FspError):
        fsp.branch_and_bound(inst, "fixed", fixed_pool=0)


@pytest.mark.parametrize("kind", ["autotuned", "learned"])
def test_graphed_kinds_reach_the_optimum(fsp, orc, kind):
    for n, m, seed in ((9, 5, 1000), (12, 8, 62), (15, 6, 67), (20, 10, 4052)):
        p = I.instance(n, m, seed)
        oc, _, ost = orc.bnb(p)
        inst = fsp.Instance(p)
        kw = {}
        if kind == "learned":
            kw["model"] = fsp.Model(2 + 2 * min(m, 15), 2, seed=1)
        for pool in (7, 4096):
            res = fsp.branch_and_bound(inst, kind, fixed_pool=pool, **kw)
            say(f"{kind} {n}x{m} pool {pool}: {res.makespan} vs {oc}, {res.nodes_bounded} nodes")
            assert res.status == 0 and res.makespan == oc
            check_schedule(orc, p, res)


def test_autotuner_picks_a_candidate_and_caches_it(fsp):
    # a shape no other test tunes: the pick is cached per (device, n, m) for
    # the process, and this short budget must not decide other tests' pools
    inst = fsp.Instance(I.instance(20, 12, 4046))
    pool, rate = fsp.autotune_pool(inst, 0.8)
    say("autotuned pool", pool, "rate", rate)
    assert pool >= 1 << 14 and (pool & (pool - 1)) == 0 and rate > 0
    assert fsp.autotune_pool(inst, 0.8) == (pool, rate)


def test_learned_kind_rejects_a_mismatched_model(fsp):
    inst = fsp.Instance(I.instance(9, 5, 1000))
    with pytest.raises(fsp.FspError):
        fsp.branch_and_bound(inst, "learned", fixed_pool=10, model=fsp.Model(22, 2))
    with pytest.raises(fsp.FspError):
        fsp.branch_and_bound(inst, "learned", fixed_pool=10)


def test_policy_samples(fsp, orc):
    """Samples logged by a search: the features are the node's depth, bound,
    prefix completion times and remaining work over the NEH makespan; the
    first target is the gap of a feasible completion to the bound (>= 0, and
    not below the best completion), the second says whether the bound
    reaches the final UB."""
    n, m = 9, 5
    p = I.instance(n, m, 1000)
    inst = fsp.Instance(p)
    x, t, res = fsp.policy_samples(inst, 500, 0.5, seed=3, kind="fixed", fixed_pool=40)
    assert res.status == 0 and 0 < x.shape[0] <= 500
    X = x.float().cpu().numpy()
    T = t.cpu().numpy()
    neh_c, _ = orc.neh(p)
    assert np.all(T[:, 0] >= 0) and set(np.unique(T[:, 1])) <= {0.0, 1.0}
    tot = p.sum(0)
    # reconstruct each node from its features: depth and bound are exact
    for r in range(min(60, len(X))):
        d = int(round(X[r, 0] * n))
        lb = X[r, 1] * neh_c  # bf16: about 3 significant digits
        assert 1 <= d < n
        # remaining work is the column total minus the prefix (same scale)
        rem = X[r, 2 + m:2 + 2 * m] * neh_c
        front = X[r, 2:2 + m] * neh_c
        assert np.all(rem <= tot * 1.01 + 1) and np.all(np.diff(front) >= -0.01 * neh_c)
        if abs(lb - res.makespan) > 0.01 * neh_c:
            assert T[r, 1] == (1.0 if lb >= res.makespan else 0.0)


@pytest.mark.parametrize("n,m,kind", [(40, 5, "adaptive"), (50, 8, "autotuned"),
                                      (80, 4, "adaptive")])
def test_larger_instances_inside_the_search(fsp, orc, n, m, kind):
    """The search on instances whose pools take the 64-bit register walk
    (33..64 jobs) or the job-mask walk (more than 64 jobs): the root bound
    equals the oracle's, and whatever the time limit leaves, the returned
    schedule is valid, no worse than NEH, and not below the smallest pending
    bound."""
    p = I.instance(n, m, 7700 + n + m)
    inst = fsp.Instance(p)
    assert inst.bound_path == ("register64" if n <= 64 else "bytes")
    say(f"{n}x{m} {kind} with a 1.5 s limit")
    res = fsp.branch_and_bound(inst, kind, time_limit=1.5)
    assert res.status in (0, 1)
    check_schedule(orc, p, res)
    assert res.root_lb == orc.lower_bound(p, [])
    neh_c, _ = orc.neh(p)
    assert res.makespan <= neh_c
    if res.status == 0:
        assert res.makespan >= res.root_lb
    else:
        assert res.root_lb <= res.open_lb <= res.makespan


@pytest.mark.parametrize("rule", ["ge", "gt"])
def test_prefilter_reaches_the_brute_force_optimum(fsp, orc, rule):
    rng = np.random.default_rng(91 if rule == "ge" else 92)
    for t in range(10):
        n, m = int(rng.integers(2, 9)), int(rng.integers(2, 8))
        p = rng.integers(1, 99, size=(n, m)).astype(np.int32)
        opt, _ = orc.brute_force(p)
        inst = fsp.Instance(p)
        for kind in ("adaptive", "autotuned"):
            res = fsp.branch_and_bound(inst, kind, prune_rule=rule, prefilter=True,
                                       **({"fixed_pool": 50} if kind == "autotuned" else {}))
            assert res.status == 0 and res.makespan == opt
            check_schedule(orc, p, res)


def test_adaptive_pool_trajectory_follows_algorithm_1(fsp, tmp_path):
    """Algorithm 1 inside a real search: the per-batch log gives the pool size
    in force and the efficiency measured; the first size is 256 threads x
    #compute units, every size doubles the previous one while the doubling
    lasts, and replaying the logged efficiencies through the schedule
    (fsp_adaptive_schedule, pinned on the CPU) gives the logged sizes."""
    import json
    inst = fsp.Instance(I.instance(20, 10, 4519))
    log = tmp_path / "adaptive.jsonl"
    res = fsp.branch_and_bound(inst, "adaptive", time_limit=3.0, log_path=str(log))
    rows = [json.loads(line) for line in open(log)]
    say(f"adaptive 20x10: {len(rows)} batches, status {res.status}")
    assert len(rows) >= 6
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    max_threads = cus * torch.cuda.get_device_properties(0).max_threads_per_multi_processor
    targets = [r["pool_target"] for r in rows]
    effs = [r["eff"] for r in rows]
    assert targets[0] == 256 * cus
    k = 1
    while k < len(targets) and targets[k] == 2 * targets[k - 1]:
        k += 1
    assert targets[k - 1] * 2 > max_threads or k == len(targets)
    assert fsp.adaptive_schedule(effs, cus, max_threads) == targets
    assert res.final_pool == targets[-1]


@pytest.mark.parametrize("kind", ["adaptive", "autotuned", "fixed"])
def test_hybrid_reaches_the_optimum(fsp, orc, kind):
    """Host threads exploring subtrees beside the device (the hybrid search):
    the optimum equals the oracle's, the schedule is valid, and the host did
    bound nodes."""
    host_total = 0
    for n, m, seed in ((12, 6, 61), (14, 7, 63), (15, 6, 64)):
        p = I.instance(n, m, seed)
        oc, _, _ = orc.bnb(p)
        inst = fsp.Instance(p)
        kw = {"fixed_pool": 50} if kind == "fixed" else {}
        res = fsp.branch_and_bound(inst, kind, host_threads=4, **kw)
        say(f"hybrid {kind} {n}x{m}: {res.makespan} vs {oc}, host nodes {res.host_nodes} "
            f"of {res.nodes_bounded}")
        assert res.status == 0 and res.makespan == oc
        check_schedule(orc, p, res)
        assert 0 <= res.host_nodes <= res.nodes_bounded
        host_total += res.host_nodes
    assert host_total > 0


@pytest.mark.parametrize("rule", ["ge", "gt"])
@pytest.mark.parametrize("packed", [True, False], ids=["packed", "one_node"])
@pytest.mark.parametrize("n,m,seed", [(9, 5, 1000), (11, 7, 71), (12, 6, 61)])
def test_bound_chosen_per_depth_counts_equal_oracle(fsp, orc, n, m, seed, rule, packed):
    """The per-depth choice of bound (Sec. VI: other lower bounds): with UB =
    the optimum, the search that gives the one-machine bound to the depths
    of a mask bounds, branches and eliminates exactly the nodes of the
    oracle's search with the same choice, in every kind, with two nodes per
    lane (packed) and one (the code of every one-node form)."""
    p = I.instance(n, m, seed)
    opt, _, _ = orc.bnb(p)
    inst = fsp.Instance(p, packed=packed)
    assert inst.bound_path == ("packed" if packed else "register")
    model = fsp.Model(2 + 2 * min(m, 15), 2, seed=seed)
    r = 0 if rule == "ge" else 1
    masks = ([1, 2, 3], [n - 1], list(range(1, n, 2)), list(range(1, n)))
    for depths in masks:
        say(f"{n}x{m} {rule}: oracle with the one-machine bound at {depths[:4]}..")
        oc, _, ost = orc.bnb_choice(p, depths, opt, r)
        assert oc == opt and ost.complete == 1
        for kind, kw in (("fixed", {"fixed_pool": 37}), ("adaptive", {}),
                         ("autotuned", {"fixed_pool": 64}),
                         ("learned", {"fixed_pool": 3000, "model": model}),
                         ("fixed", {"fixed_pool": 37, "prefilter": True})):
            res = fsp.branch_and_bound(inst, kind, ub=opt, prune_rule=rule, bound_choice=2,
                                       lb1_depths=depths, **kw)
            say(f"{n}x{m} {rule} lb1 at {depths[:4]}.. {kind}: {res.nodes_bounded} vs "
                f"{ost.nodes_bounded}")
            assert res.makespan == opt and res.found == 0 and res.status == 0
            assert res.nodes_bounded == ost.nodes_bounded
            assert res.nodes_branched == ost.nodes_branched
            assert res.leaves == ost.leaves
            assert res.nodes_pruned == ost.nodes_pruned


def test_autotuned_bound_choice_reaches_the_optimum(fsp, orc):
    """fsp_autotune_bounds: the depths it picks are within 1..n-1, no two
    adjacent, the same on a second call (cached); searches with the choice
    from NEH return the oracle's optimum with a valid schedule; the counts
    behind the choice are consistent (the pair bound eliminates every node
    the one-machine bound eliminates)."""
    for n, m, seed in ((12, 6, 61), (14, 7, 63), (20, 10, 4501)):
        p = I.instance(n, m, seed)
        inst = fsp.Instance(p)
        depths = fsp.autotune_bounds(inst, 0.5)
        say(f"{n}x{m}: one-machine bound at depths {depths}")
        assert all(1 <= d <= n - 1 for d in depths)
        assert all(b - a >= 2 for a, b in zip(depths, depths[1:]))
        assert fsp.autotune_bounds(inst) == depths
        res, st = fsp.depth_stats(inst, "autotuned", time_limit=0.5)
        assert (st[1] <= st[2]).all() and (st[2] <= st[0]).all()
        assert int(st[0].sum()) <= res.nodes_bounded
        assert st[0][n:].sum() == 0 and st[0][0] == 0
        if n <= 14:
            oc, _, _ = orc.bnb(p)
            for kind in ("adaptive", "autotuned"):
                res = fsp.branch_and_bound(inst, kind, bound_choice=1)
                assert res.status == 0 and res.makespan == oc
                check_schedule(orc, p, res)
