"""Python binding of libfsp (the C ABI declared in include/fsp.h).

Argument marshalling only: every step of the bounding path runs in the HIP
kernels of ``libfsp.so``.  torch provides device memory and streams.  The
library is loaded after ``import torch`` so that both share one HIP runtime
(torch's ``libamdhip64.so.7``); if ``libfsp.so`` has not been built, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfsp.so")

FSP_OK = 0
FSP_EINVAL = -1
FSP_ENOMEM = -2
FSP_EDEVICE = -3
FSP_EUNSUPPORTED = -4
FSP_ESCRATCH = -5
FSP_LB_INVALID = -1

_lib = None


LOAD_ONE_NODE_PER_LANE = 1  # FSP_LOAD_ONE_NODE_PER_LANE
LOAD_JOB_MASKS = 2  # FSP_LOAD_JOB_MASKS


class FspError(RuntimeError):
    def __init__(self, rc: int, what: str):
        self.rc = rc
        super().__init__(f"{what}: {status_string(rc)} ({rc})")


class _Nodes(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("stride", ctypes.c_int32)]


class _Segment(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("stride", ctypes.c_int32), ("count", ctypes.c_int64),
                ("lb_out", ctypes.c_void_p)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("one_node_per_lane", ctypes.c_int32), ("job_masks", ctypes.c_int32)]


POOL_KINDS = {"fixed": 0, "adaptive": 1, "autotuned": 2, "learned": 3}
PRUNE_RULES = {"ge": 0, "gt": 1}


class _Policy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nb_iterations", ctypes.c_int32),
                ("fixed_pool", ctypes.c_int64), ("max_pool", ctypes.c_int64),
                ("time_limit_s", ctypes.c_double), ("prune_rule", ctypes.c_int32),
                ("prefilter", ctypes.c_int32), ("model", ctypes.c_void_p),
                ("log_path", ctypes.c_char_p), ("host_threads", ctypes.c_int32),
                ("bound_choice", ctypes.c_int32), ("lb1_depths", ctypes.c_uint32 * 8)]


class _Result(ctypes.Structure):
    _fields_ = [("makespan", ctypes.c_int32), ("found", ctypes.c_int32),
                ("perm", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("root_lb", ctypes.c_int32), ("nodes_bounded", ctypes.c_int64),
                ("nodes_branched", ctypes.c_int64), ("nodes_pruned", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("pools", ctypes.c_int64),
                ("t_found_s", ctypes.c_double), ("t_total_s", ctypes.c_double),
                ("final_pool", ctypes.c_int64), ("t_search_s", ctypes.c_double),
                ("open_lb", ctypes.c_int32), ("proof_pools", ctypes.c_int32),
                ("host_nodes", ctypes.c_int64)]


def lib() -> ctypes.CDLL:
    """The loaded library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1206_4973_amd.build`"
        )
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.fsp_status_string.argtypes = [i32]
    L.fsp_status_string.restype = ctypes.c_char_p
    L.fsp_load_instance.argtypes = [P, i32, i32, ctypes.POINTER(P)]
    L.fsp_load_instance.restype = ctypes.c_int
    L.fsp_load_instance_ex.argtypes = [P, i32, i32, i32, ctypes.POINTER(P)]
    L.fsp_load_instance_ex.restype = ctypes.c_int
    L.fsp_free_instance.argtypes = [P]
    L.fsp_free_instance.restype = ctypes.c_int
    L.fsp_instance_info.argtypes = [P, P, P, P]
    L.fsp_instance_info.restype = ctypes.c_int
    L.fsp_bound_pool_one_machine.argtypes = [ctypes.POINTER(_Nodes), i64, P, P]
    L.fsp_bound_pool_one_machine.restype = ctypes.c_int
    L.fsp_bound_pool_noalloc.argtypes = [ctypes.POINTER(_Nodes), i64, P, P]
    L.fsp_bound_pool_noalloc.restype = ctypes.c_int
    L.fsp_noalloc_max_count.argtypes = [i32]
    L.fsp_noalloc_max_count.restype = i64
    L.fsp_instance_path.argtypes = [P, P]
    L.fsp_instance_path.restype = ctypes.c_int
    L.fsp_bound_pool.argtypes = [ctypes.POINTER(_Nodes), i64, P, P]
    L.fsp_bound_pool.restype = ctypes.c_int
    L.fsp_branch_and_bound.argtypes = [P, ctypes.POINTER(_Policy), i32,
                                       ctypes.POINTER(_Result)]
    L.fsp_branch_and_bound.restype = ctypes.c_int
    L.fsp_neh.argtypes = [P, P, ctypes.POINTER(i32)]
    L.fsp_neh.restype = ctypes.c_int
    L.fsp_batch_create.argtypes = [ctypes.POINTER(_Segment), i32,
                                   ctypes.POINTER(_BatchConfig), ctypes.POINTER(P)]
    L.fsp_batch_create.restype = ctypes.c_int
    L.fsp_batch_launch.argtypes = [P, P]
    L.fsp_batch_launch.restype = ctypes.c_int
    L.fsp_batch_replay.argtypes = [P, P]
    L.fsp_batch_replay.restype = ctypes.c_int
    L.fsp_batch_info.argtypes = [P, P, P, P, P]
    L.fsp_batch_info.restype = ctypes.c_int
    L.fsp_batch_paths.argtypes = [P, P, i32, P]
    L.fsp_batch_paths.restype = ctypes.c_int
    L.fsp_batch_free.argtypes = [P]
    L.fsp_batch_free.restype = ctypes.c_int
    L.fsp_bound_batch.argtypes = [ctypes.POINTER(_Segment), i32, P]
    L.fsp_bound_batch.restype = ctypes.c_int
    L.fsp_autotune_pool.argtypes = [P, ctypes.c_double, ctypes.POINTER(i64),
                                    ctypes.POINTER(ctypes.c_double)]
    L.fsp_autotune_pool.restype = ctypes.c_int
    L.fsp_adaptive_schedule.argtypes = [i32, i32, i64, i64, P, i32, P]
    L.fsp_adaptive_schedule.restype = ctypes.c_int
    L.fsp_autotune_bounds.argtypes = [P, ctypes.c_double, P]
    L.fsp_autotune_bounds.restype = ctypes.c_int
    L.fsp_bound_choice_rule.argtypes = [i32, P, P, P, P]
    L.fsp_bound_choice_rule.restype = ctypes.c_int
    L.fsp_depth_stats.argtypes = [P, ctypes.POINTER(_Policy), i32, P, ctypes.POINTER(_Result)]
    L.fsp_depth_stats.restype = ctypes.c_int
    L.fsp_policy_samples.argtypes = [P, ctypes.POINTER(_Policy), i32, i64, ctypes.c_double,
                                     ctypes.c_uint64, P, P, ctypes.POINTER(i64),
                                     ctypes.POINTER(_Result)]
    L.fsp_policy_samples.restype = ctypes.c_int
    L.fsp_model_create.argtypes = [i32, i32, i32, ctypes.c_uint64, ctypes.POINTER(P)]
    L.fsp_model_create.restype = ctypes.c_int
    L.fsp_model_free.argtypes = [P]
    L.fsp_model_free.restype = ctypes.c_int
    L.fsp_model_param_count.argtypes = []
    L.fsp_model_param_count.restype = i64
    L.fsp_model_set_trained_jobs.argtypes = [P, i32]
    L.fsp_model_set_trained_jobs.restype = ctypes.c_int
    for name in ("fsp_model_set_params", "fsp_model_get_params", "fsp_model_get_grads"):
        getattr(L, name).argtypes = [P, P, i64]
        getattr(L, name).restype = ctypes.c_int
    L.fsp_model_forward.argtypes = [P, P, i64, P, P]
    L.fsp_model_forward.restype = ctypes.c_int
    L.fsp_model_backward.argtypes = [P, P, i64, P, P, i32, P]
    L.fsp_model_backward.restype = ctypes.c_int
    L.fsp_model_adam_step.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, P]
    L.fsp_model_adam_step.restype = ctypes.c_int
    L.fsp_model_train_step.argtypes = [P, P, P, i64, ctypes.c_float,
                                       ctypes.POINTER(ctypes.c_float), P]
    L.fsp_model_train_step.restype = ctypes.c_int
    _lib = L
    return L


def status_string(rc: int) -> str:
    return lib().fsp_status_string(int(rc)).decode()


def _check(rc: int, what: str) -> None:
    if rc != FSP_OK:
        raise FspError(rc, what)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Instance:
    """An instance loaded on the current device (fsp_load_instance_ex).
    packed=False keeps an instance that qualifies for the two-nodes-per-lane
    16-bit form on the one-node-per-lane 32-bit form (same bounds)."""

    def __init__(self, p, packed: bool = True, job_masks: bool = False):
        if isinstance(p, torch.Tensor):
            p = p.detach().cpu().numpy()
        p = np.ascontiguousarray(p, dtype=np.int32)
        if p.ndim != 2:
            raise ValueError("p must be a [n, m] matrix")
        self.p = p
        self.n, self.m = int(p.shape[0]), int(p.shape[1])
        h = ctypes.c_void_p()
        flags = (0 if packed else LOAD_ONE_NODE_PER_LANE) | (LOAD_JOB_MASKS if job_masks else 0)
        _check(lib().fsp_load_instance_ex(p.ctypes.data_as(ctypes.c_void_p), self.n, self.m,
                                          flags, ctypes.byref(h)), "fsp_load_instance_ex")
        self._h = h
        dev = ctypes.c_int32()
        _check(lib().fsp_instance_info(h, None, None, ctypes.byref(dev)), "fsp_instance_info")
        self.device = torch.device("cuda", dev.value)

    @property
    def bound_path(self) -> str:
        """Form of the bounding walk used for this instance: "register",
        "packed" (two nodes per lane, 16-bit), "register64" (33..64 jobs),
        "bytes" (n > 64) or "masks" (n > 64, loaded with job_masks=True)."""
        v = ctypes.c_int32(0)
        _check(lib().fsp_instance_path(self.handle, ctypes.byref(v)), "fsp_instance_path")
        return {0: "register", 1: "packed", 2: "masks", 3: "register64", 4: "bytes"}[v.value]

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("instance is closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().fsp_free_instance(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bound_pool(self, nodes: torch.Tensor, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """Bounds of a ``uint8 [count, stride]`` device pool (fsp_bound_pool).

        Asynchronous on ``stream`` (default: torch's current stream)."""
        return _bound_call(self, "fsp_bound_pool", nodes, out, stream)

    def bound_pool_noalloc(self, nodes: torch.Tensor, out: torch.Tensor,
                           stream=None) -> torch.Tensor:
        """fsp_bound_pool without any device allocation (fsp_bound_pool_noalloc):
        ``out`` must be given; pools above ``noalloc_max_count`` raise."""
        if out is None:
            raise ValueError("bound_pool_noalloc needs a caller-provided out tensor")
        return _bound_call(self, "fsp_bound_pool_noalloc", nodes, out, stream)

    @property
    def noalloc_max_count(self) -> int:
        """Largest pool bound_pool_noalloc accepts: the fixed scratch limits
        only the job-mask walk; every other walk takes no scratch."""
        if self.bound_path != "masks":
            return (1 << 63) - 1
        return int(lib().fsp_noalloc_max_count(self.n))

    def bound_pool_one_machine(self, nodes: torch.Tensor, out: torch.Tensor | None = None,
                               stream=None) -> torch.Tensor:
        """One-machine bounds of a ``uint8 [count, stride]`` device pool
        (fsp_bound_pool_one_machine); asynchronous on ``stream``."""
        return _bound_call(self, "fsp_bound_pool_one_machine", nodes, out, stream)


def _bound_call(inst, fn_name, nodes, out, stream):
    if nodes.dtype != torch.uint8 or nodes.dim() != 2 or not nodes.is_cuda:
        raise ValueError("nodes must be a uint8 [count, stride] device tensor")
    if nodes.stride(1) != 1:
        raise ValueError("records must be contiguous")
    count, stride = int(nodes.shape[0]), int(nodes.stride(0))
    if out is None:
        out = torch.empty(count, dtype=torch.int32, device=nodes.device)
    if out.dtype != torch.int32 or out.numel() < count or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 device tensor of >= count")
    desc = _Nodes(inst.handle.value, nodes.data_ptr(), stride)
    _check(getattr(lib(), fn_name)(ctypes.byref(desc), count,
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           fn_name)
    return out


class Result:
    """Outcome of fsp_branch_and_bound (see fsp_result in include/fsp.h)."""

    def __init__(self, r: _Result, perm: np.ndarray):
        for name, _ in _Result._fields_:
            if name != "perm":
                setattr(self, name, getattr(r, name))
        self.perm = perm

    def __repr__(self):
        keys = ("makespan", "found", "status", "root_lb", "nodes_bounded", "nodes_branched",
                "nodes_pruned", "leaves", "pools", "t_found_s", "t_total_s", "t_search_s",
                "final_pool", "open_lb", "proof_pools", "host_nodes")
        return "Result(" + ", ".join(f"{k}={getattr(self, k)}" for k in keys) + ")"


def make_policy(kind: str = "adaptive", *, fixed_pool: int = 0, max_pool: int = 0,
                nb_iterations: int = 10, time_limit: float | None = None,
                prune_rule: str = "ge", model=None, log_path: str | None = None,
                prefilter: bool = False, host_threads: int = 0,
                bound_choice: int = 0, lb1_depths=None) -> _Policy:
    """The search policy (fsp_pool_policy).  bound_choice: 0 the two-machine
    bound at every depth; 1 the depths fsp_autotune_bounds picks take the
    one-machine bound; 2 the depths in `lb1_depths` (an iterable of depths)
    take it."""
    pol = _Policy()
    pol.kind = POOL_KINDS[kind]
    pol.nb_iterations = int(nb_iterations)
    pol.fixed_pool = int(fixed_pool)
    pol.max_pool = int(max_pool)
    pol.time_limit_s = float(time_limit) if time_limit else 0.0
    pol.prune_rule = PRUNE_RULES[prune_rule]
    pol.prefilter = 1 if prefilter else 0
    pol.model = ctypes.c_void_p(model.handle.value) if model is not None else None
    pol.log_path = log_path.encode() if log_path else None
    pol.host_threads = int(host_threads)
    pol.bound_choice = int(bound_choice)
    for d in (lb1_depths or ()):
        pol.lb1_depths[int(d) >> 5] |= 1 << (int(d) & 31)
    return pol


def branch_and_bound(inst: Instance, kind: str = "adaptive", ub: int | None = None,
                     **policy) -> Result:
    """Exact minimum makespan by device-resident B&B (fsp_branch_and_bound)."""
    pol = make_policy(kind, **policy)
    perm = np.zeros(max(inst.n, 1), dtype=np.uint8)
    res = _Result()
    res.perm = perm.ctypes.data_as(ctypes.c_void_p).value
    _check(lib().fsp_branch_and_bound(inst.handle, ctypes.byref(pol),
                                      int(ub) if ub else 0, ctypes.byref(res)),
           "fsp_branch_and_bound")
    return Result(res, perm[:inst.n].copy())


def _mask_depths(words) -> list:
    return [32 * w + b for w in range(8) for b in range(32) if (int(words[w]) >> b) & 1]


def autotune_bounds(inst: Instance, budget_s: float = 0.0) -> list:
    """Depths that fsp_autotune_bounds gives the one-machine bound (cached
    per shape)."""
    mask = (ctypes.c_uint32 * 8)()
    _check(lib().fsp_autotune_bounds(inst.handle, float(budget_s), mask), "fsp_autotune_bounds")
    return _mask_depths(mask)


def bound_choice_rule(n: int, total, elim1, elim2) -> list:
    """Depths that fsp_bound_choice_rule gives the one-machine bound for the
    per-depth counts (host only)."""
    arrs = [np.zeros(256, dtype=np.uint32) for _ in range(3)]
    for a, v in zip(arrs, (total, elim1, elim2)):
        v = np.asarray(v, dtype=np.uint32)
        a[:len(v)] = v
    mask = (ctypes.c_uint32 * 8)()
    _check(lib().fsp_bound_choice_rule(int(n), *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs],
                                       mask), "fsp_bound_choice_rule")
    return _mask_depths(mask)


def depth_stats(inst: Instance, kind: str = "adaptive", ub: int | None = None, **policy):
    """(Result, counts [3][256]) of fsp_depth_stats: per depth, bounded nodes
    with jobs left and those the one-machine and the two-machine bound
    eliminate."""
    pol = make_policy(kind, **policy)
    perm = np.zeros(max(inst.n, 1), dtype=np.uint8)
    res = _Result()
    res.perm = perm.ctypes.data_as(ctypes.c_void_p).value
    st = np.zeros((3, 256), dtype=np.uint32)
    _check(lib().fsp_depth_stats(inst.handle, ctypes.byref(pol), int(ub) if ub else 0,
                                 st.ctypes.data_as(ctypes.c_void_p), ctypes.byref(res)),
           "fsp_depth_stats")
    return Result(res, perm[:inst.n].copy()), st


def autotune_pool(inst: Instance, budget_s: float = 0.0):
    """(pool size, nodes/s) picked by fsp_autotune_pool for this shape (cached)."""
    pool, rate = ctypes.c_int64(), ctypes.c_double()
    _check(lib().fsp_autotune_pool(inst.handle, float(budget_s), ctypes.byref(pool),
                                   ctypes.byref(rate)), "fsp_autotune_pool")
    return int(pool.value), float(rate.value)


def adaptive_schedule(efficiency, cus: int, max_threads: int, max_pool: int = 0,
                      threads_per_block: int = 256) -> list:
    """Pool targets Algorithm 1 sets batch by batch for the given measured
    efficiencies (fsp_adaptive_schedule; host only)."""
    eff = np.ascontiguousarray(efficiency, dtype=np.float64)
    out = np.zeros(len(eff), dtype=np.int64)
    _check(lib().fsp_adaptive_schedule(int(threads_per_block), int(cus), int(max_threads),
                                       int(max_pool), eff.ctypes.data_as(ctypes.c_void_p),
                                       len(eff), out.ctypes.data_as(ctypes.c_void_p)),
           "fsp_adaptive_schedule")
    return [int(x) for x in out]


def policy_samples(inst: Instance, max_samples: int, sample_prob: float, seed: int = 0,
                   kind: str = "adaptive", ub: int | None = None, **policy):
    """Training samples logged by a search (fsp_policy_samples).

    Returns (x bf16 [k, 32], target fp32 [k, 2], Result), device tensors."""
    pol = make_policy(kind, **policy)
    x = torch.empty((max_samples, 32), dtype=torch.bfloat16, device="cuda")
    t = torch.empty((max_samples, 2), dtype=torch.float32, device="cuda")
    nout = ctypes.c_int64()
    perm = np.zeros(max(inst.n, 1), dtype=np.uint8)
    res = _Result()
    res.perm = perm.ctypes.data_as(ctypes.c_void_p).value
    _check(lib().fsp_policy_samples(inst.handle, ctypes.byref(pol), int(ub) if ub else 0,
                                    int(max_samples), float(sample_prob), ctypes.c_uint64(seed),
                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                    ctypes.byref(nout), ctypes.byref(res)),
           "fsp_policy_samples")
    k = int(nout.value)
    return x[:k], t[:k], Result(res, perm[:inst.n].copy())


def neh(inst: Instance):
    """(makespan, permutation) of the NEH insertion heuristic (fsp_neh)."""
    perm = np.zeros(inst.n, dtype=np.uint8)
    c = ctypes.c_int32()
    _check(lib().fsp_neh(inst.handle, perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(c)),
           "fsp_neh")
    return int(c.value), perm


def _segments(items):
    segs = (_Segment * max(1, len(items)))()
    outs = []
    for i, (inst, nodes, out) in enumerate(items):
        if nodes.dtype != torch.uint8 or nodes.dim() != 2 or not nodes.is_cuda:
            raise ValueError("nodes must be a uint8 [count, stride] device tensor")
        count = int(nodes.shape[0])
        if out is None:
            out = torch.empty(count, dtype=torch.int32, device=nodes.device)
        segs[i].inst = inst.handle.value
        segs[i].data = nodes.data_ptr()
        segs[i].stride = int(nodes.stride(0)) if count > 0 else int(nodes.shape[1])
        segs[i].count = count
        segs[i].lb_out = out.data_ptr()
        outs.append(out)
    return segs, outs


class Batch:
    """A batch of (instance, pool) segments bounded in one persistent launch
    (fsp_batch_create / fsp_batch_launch / fsp_batch_replay).

    ``items``: list of (Instance, uint8 [count, stride] device tensor,
    int32 [count] device tensor or None).  The tensors must stay alive (and
    keep their storage) as long as the batch is used.  The keywords are the
    fields of fsp_batch_config: ``packed=False`` sets one_node_per_lane,
    ``job_masks=True`` puts segments above 64 jobs on the job masks."""

    def __init__(self, items, blocks_per_cu: int = 0, autotune: bool = False,
                 packed: bool = True, job_masks: bool = False):
        self._keep = [(i, n) for i, n, _ in items]
        self.nsegs = len(items)
        segs, self.outs = _segments(items)
        cfg = _BatchConfig()
        cfg.blocks_per_cu = int(blocks_per_cu)
        cfg.autotune = 1 if autotune else 0
        cfg.one_node_per_lane = 0 if packed else 1
        cfg.job_masks = 1 if job_masks else 0
        h = ctypes.c_void_p()
        _check(lib().fsp_batch_create(segs, len(items), ctypes.byref(cfg), ctypes.byref(h)),
               "fsp_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().fsp_batch_launch(self._h, _stream_handle(stream)), "fsp_batch_launch")
        return self.outs

    def replay(self, stream=None):
        _check(lib().fsp_batch_replay(self._h, _stream_handle(stream)), "fsp_batch_replay")
        return self.outs

    def info(self) -> dict:
        tiles, grid = ctypes.c_int64(), ctypes.c_int32()
        ks, fs = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fsp_batch_info(self._h, ctypes.byref(tiles), ctypes.byref(grid),
                                    ctypes.byref(ks), ctypes.byref(fs)), "fsp_batch_info")
        return {"tiles": tiles.value, "grid": grid.value, "kernel_segments": ks.value,
                "fallback_segments": fs.value}

    def paths(self):
        """(walk form name of every segment, or None; workgroups per CU)."""
        arr = (ctypes.c_int32 * max(1, self.nsegs))()
        bpc = ctypes.c_int32()
        _check(lib().fsp_batch_paths(self._h, arr, self.nsegs, ctypes.byref(bpc)),
               "fsp_batch_paths")
        names = {0: "register", 1: "packed", 2: "masks", 3: "register64", 4: "bytes"}
        return [names.get(arr[i]) for i in range(self.nsegs)], bpc.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fsp_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bound_batch(items, stream=None):
    """One-shot batch (fsp_bound_batch): returns the bound tensors."""
    segs, outs = _segments(items)
    _check(lib().fsp_bound_batch(segs, len(items), _stream_handle(stream)), "fsp_bound_batch")
    return outs


class Model:
    """The pool-policy network (fsp_model_*): 32 -> 128 -> 128 -> outputs."""

    def __init__(self, in_features: int = 22, outputs: int = 2, seed: int = 0,
                 hidden: int = 128):
        h = ctypes.c_void_p()
        _check(lib().fsp_model_create(int(in_features), int(hidden), int(outputs),
                                      ctypes.c_uint64(seed), ctypes.byref(h)),
               "fsp_model_create")
        self._h = h
        self.in_features, self.outputs = int(in_features), int(outputs)
        self.nparams = int(lib().fsp_model_param_count())

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fsp_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().fsp_model_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                          self.nparams), "fsp_model_get_params")
        return out

    def set_params(self, p: np.ndarray) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().fsp_model_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                          len(p)), "fsp_model_set_params")

    def set_trained_jobs(self, n: int) -> None:
        """Job count of the training instances (gates the learned search's
        switch to proof pools; 0: unknown)."""
        _check(lib().fsp_model_set_trained_jobs(self._h, int(n)), "fsp_model_set_trained_jobs")

    def grads(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().fsp_model_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                         self.nparams), "fsp_model_get_grads")
        return out

    @staticmethod
    def _x(x: torch.Tensor) -> torch.Tensor:
        if x.dtype != torch.bfloat16 or x.dim() != 2 or x.shape[1] != 32 or not x.is_cuda:
            raise ValueError("x must be a bfloat16 [N, 32] device tensor")
        return x.contiguous()

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        x = self._x(x)
        y = torch.empty((x.shape[0], self.outputs), dtype=torch.float32, device=x.device)
        _check(lib().fsp_model_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                       ctypes.c_void_p(y.data_ptr()), _stream_handle(stream)),
               "fsp_model_forward")
        return y

    def backward(self, x: torch.Tensor, dy: torch.Tensor, want_dx: bool = False,
                 accumulate: bool = False, stream=None):
        x = self._x(x)
        dy = dy.contiguous().float()
        dx = torch.empty((x.shape[0], 32), dtype=torch.float32, device=x.device) if want_dx else None
        _check(lib().fsp_model_backward(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                        ctypes.c_void_p(dy.data_ptr()),
                                        ctypes.c_void_p(dx.data_ptr()) if dx is not None else None,
                                        1 if accumulate else 0, _stream_handle(stream)),
               "fsp_model_backward")
        return dx

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                  weight_decay: float = 0.0, stream=None) -> None:
        _check(lib().fsp_model_adam_step(self._h, lr, beta1, beta2, eps, weight_decay,
                                         _stream_handle(stream)), "fsp_model_adam_step")

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float, stream=None) -> float:
        x = self._x(x)
        target = target.contiguous().float()
        loss = ctypes.c_float()
        _check(lib().fsp_model_train_step(self._h, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(target.data_ptr()), x.shape[0], lr,
                                          ctypes.byref(loss), _stream_handle(stream)),
               "fsp_model_train_step")
        return float(loss.value)
