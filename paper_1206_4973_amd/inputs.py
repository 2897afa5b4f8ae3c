"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

Holds no arithmetic of the method: it only draws processing-time matrices and
node records.  The workloads stand in for Taillard's flow-shop benchmark (the
paper's Sec. V.A), which is not reproduced: instances keep its shape classes
(n in {20, 50, 100, 200} jobs x m in {5, 10, 20} machines) and draw integer
processing times uniformly in [1, 99].

Node record layout (shared with the C ABI): ``uint8[stride]`` with byte 0 the
depth d (number of scheduled jobs) and bytes 1..d the scheduled prefix (job ids
in schedule order).  Bytes after the prefix are zero.  The default stride is
n+1 rounded up to a multiple of 16, so every record is 16-byte aligned.
"""
from __future__ import annotations

import numpy as np


def instance(n: int, m: int, seed: int, lo: int = 1, hi: int = 99) -> np.ndarray:
    """Processing times p[j][k] (job j, machine k), int32 uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, m), dtype=np.int32)


def node_stride(n: int) -> int:
    return ((n + 1 + 15) // 16) * 16


def records(prefixes, n: int, stride: int | None = None) -> np.ndarray:
    """Pack a list of prefixes (sequences of job ids) into node records."""
    stride = node_stride(n) if stride is None else stride
    out = np.zeros((len(prefixes), stride), dtype=np.uint8)
    for i, pre in enumerate(prefixes):
        out[i, 0] = len(pre)
        out[i, 1:1 + len(pre)] = np.asarray(pre, dtype=np.uint8)
    return out


def random_pool(n: int, count: int, dlo: int, dhi: int, seed: int,
                stride: int | None = None, chunk: int = 1 << 16) -> np.ndarray:
    """``count`` random nodes: depth uniform in [dlo, dhi], prefix = the first d
    entries of a uniformly random permutation of the n jobs.

    Drawn chunk by chunk (each chunk from its own child of ``seed``) so that
    million-node pools need little memory; the result depends only on the
    arguments.
    """
    stride = node_stride(n) if stride is None else stride
    assert stride >= n + 1 and 0 <= dlo <= dhi <= n
    out = np.zeros((count, stride), dtype=np.uint8)
    nchunks = (count + chunk - 1) // chunk
    seqs = np.random.SeedSequence(seed).spawn(max(nchunks, 1))
    base = np.arange(n, dtype=np.uint8)
    cols = np.arange(n)
    for c in range(nchunks):
        rng = np.random.default_rng(seqs[c])
        b, e = c * chunk, min(count, (c + 1) * chunk)
        k = e - b
        d = rng.integers(dlo, dhi + 1, size=k)
        perm = rng.permuted(np.broadcast_to(base, (k, n)), axis=1)
        keep = cols[None, :] < d[:, None]
        out[b:e, 0] = d.astype(np.uint8)
        out[b:e, 1:1 + n] = np.where(keep, perm, 0).astype(np.uint8)
    return out


def sibling_pool(n: int, parents: int, dlo: int, dhi: int, seed: int,
                 stride: int | None = None) -> np.ndarray:
    """A branching-shaped pool: ``parents`` random prefixes (depth uniform in
    [dlo, dhi], dhi < n), each followed by all of its children in ascending
    order of the appended job (the layout a branching step produces)."""
    stride = node_stride(n) if stride is None else stride
    par = random_pool(n, parents, dlo, dhi, seed, stride)
    recs = []
    for r in par:
        d = int(r[0])
        pre = r[1:1 + d]
        used = np.zeros(n, dtype=bool)
        used[pre] = True
        for j in range(n):
            if not used[j]:
                c = np.zeros(stride, dtype=np.uint8)
                c[0] = d + 1
                c[1:1 + d] = pre
                c[1 + d] = j
                recs.append(c)
    return np.stack(recs) if recs else np.zeros((0, stride), np.uint8)
