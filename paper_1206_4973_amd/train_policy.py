"""Train the pool-policy network on samples that branch-and-bound runs log.

    python -m paper_1206_4973_amd.train_policy --out paper_1206_4973_amd/policy_20x10.npz

1. For every training instance (20 jobs x 10 machines, seeds 4000..4199 by
   default) a plain adaptive search runs for a short time limit and logs a
   random sample of the children that survive elimination
   (fsp_policy_samples): the network input of each node and its two targets
   (completion gap of a suffix-NEH completion, and whether the final UB would
   have eliminated it).
2. The network (fsp_model_*) is trained on all samples with its own forward,
   backward and Adam kernels; torch only provides device memory and the
   shuffling permutation.
3. The parameters are saved with the shapes needed to rebuild the model.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import fsp, inputs


def parse_seeds(text: str) -> list[int]:
    out = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        elif part:
            out.append(int(part))
    return out


def collect(seeds, n, m, time_limit, max_samples, prob, log=print):
    xs, ts = [], []
    t0 = time.time()
    for i, s in enumerate(seeds):
        inst = fsp.Instance(inputs.instance(n, m, s))
        x, t, res = fsp.policy_samples(inst, max_samples, prob, seed=s, kind="adaptive",
                                       time_limit=time_limit)
        xs.append(x.clone())
        ts.append(t.clone())
        inst.close()
        if (i + 1) % 20 == 0 or i + 1 == len(seeds):
            log(f"  samples from {i + 1}/{len(seeds)} instances: "
                f"{sum(len(a) for a in xs)} ({time.time() - t0:.1f} s)")
    return torch.cat(xs), torch.cat(ts)


def train(x, t, in_features, epochs, batch, lr, seed, log=print):
    torch.manual_seed(seed)
    model = fsp.Model(in_features, 2, seed=seed)
    n = x.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(n, device=x.device)
        tot, cnt = 0.0, 0
        for b in range(0, n - batch + 1, batch):
            idx = perm[b:b + batch]
            tot += model.train_step(x[idx].contiguous(), t[idx].contiguous(), lr)
            cnt += 1
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: mean batch loss {tot / max(cnt, 1):.5f}")
    return model


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--seeds", default="4000-4199")
    ap.add_argument("--time-limit", type=float, default=0.3)
    ap.add_argument("--samples", type=int, default=4000, help="per instance, at most")
    ap.add_argument("--prob", type=float, default=0.02)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    seeds = parse_seeds(args.seeds)
    print(f"collecting samples from {len(seeds)} instances {args.n}x{args.m}", flush=True)
    x, t = collect(seeds, args.n, args.m, args.time_limit, args.samples, args.prob,
                   log=lambda s: print(s, flush=True))
    in_features = 2 + 2 * min(args.m, 15)
    print(f"training on {x.shape[0]} samples", flush=True)
    model = train(x, t, in_features, args.epochs, args.batch, args.lr, args.seed,
                  log=lambda s: print(s, flush=True))
    meta = {"in_features": in_features, "outputs": 2, "n": args.n, "m": args.m,
            "seeds": args.seeds, "samples": int(x.shape[0]), "epochs": args.epochs,
            "time_limit": args.time_limit, "prob": args.prob}
    np.savez(args.out, params=model.params(), meta=json.dumps(meta))
    print("saved", args.out, json.dumps(meta), flush=True)
    return 0


def load(path: str) -> fsp.Model:
    """Rebuild a trained model saved by this script."""
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    model = fsp.Model(meta["in_features"], meta["outputs"])
    model.set_params(z["params"])
    model.set_trained_jobs(int(meta.get("n", 0)))
    return model


if __name__ == "__main__":
    sys.exit(main())
