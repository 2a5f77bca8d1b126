"""Open-loop driver of the serving loop (fks_server_*): a Poisson stream of build and
lookup requests replayed in real time against one FksServer, with the latency of
every request (completion minus submission) and the sustained query rate."""
from __future__ import annotations

import time

import numpy as np

from . import fks, workloads


class Workload:
    """Requests of a stream with their device data made ahead of time.

    Build request b gets the keys mix(base_b + [0, n_b)) with disjoint index ranges per
    map; lookup needles are half keys of the target map and half mix() of indices no map
    uses, so hit/miss is known exactly.  The target of a lookup is chosen among the maps
    submitted before it (prebuilt ones included)."""

    def __init__(self, requests, prebuilt_sizes, seed: int, device):
        import torch
        self.requests = requests
        self.device = device
        rng = np.random.Generator(np.random.PCG64(seed))
        self.maps = []          # (keys tensor, vals tensor, seed, n, index base)
        base = 0
        for n in prebuilt_sizes:
            self._add_map(int(n), base, int(rng.integers(1 << 62)))
            base += int(n)
        self.n_prebuilt = len(prebuilt_sizes)
        self.plan = []          # per request: ('build', map index) or ('lookup', map, q, expect)
        miss_base = 1 << 62
        for r in requests:
            if r["kind"] == "build":
                self._add_map(r["size"], base, r["seed"])
                base += r["size"]
                self.plan.append(("build", len(self.maps) - 1))
            else:
                avail = len(self.maps)
                tgt = min(int(r["pick"] * avail), avail - 1)
                keys, _, _, n, kb = self.maps[tgt]
                m = r["size"]
                nh = m // 2
                sub = np.random.Generator(np.random.PCG64(r["seed"]))
                hit_idx = sub.integers(0, n, size=nh)
                miss_idx = miss_base + np.arange(m - nh, dtype=np.uint64)
                miss_base += m - nh
                idx = np.concatenate([kb + hit_idx.astype(np.uint64), miss_idx])
                expect = np.concatenate([np.ones(nh, np.uint8), np.zeros(m - nh, np.uint8)])
                perm = sub.permutation(m)
                idx, expect = idx[perm], expect[perm]
                q = workloads.mix_keys_torch(torch.from_numpy(idx.view(np.int64)).to(device))
                vals_expect = np.where(expect == 1, (idx - np.uint64(kb)).astype(np.uint32), 0xFFFFFFFF)
                self.plan.append(("lookup", tgt, q, torch.from_numpy(expect).to(device),
                                  torch.from_numpy(vals_expect.astype(np.uint32).view(np.int32)).to(device)))

    def _add_map(self, n, base, seed):
        import torch
        idx = torch.arange(base, base + n, dtype=torch.int64, device=self.device)
        keys = workloads.mix_keys_torch(idx)
        vals = torch.arange(n, dtype=torch.int32, device=self.device)
        self.maps.append((keys, vals, seed, n, base))


def run(wl: Workload, budget_bytes: int, rate_scale: float = 1.0, graphs: bool = True, closed_loop=False):
    """Replay the stream (arrival times divided by rate_scale; closed_loop submits all at
    once).  Returns a result dict with per-kind p50/p99 latency and throughput, and the
    per-request outputs for checking."""
    import torch
    srv = fks.FksServer(budget_bytes, graphs=graphs)
    map_ids = []
    for keys, vals, seed, n, _ in wl.maps[:wl.n_prebuilt]:
        _, mid = srv.submit_build(keys, vals, seed)
        map_ids.append(mid)
    srv.wait_all()
    n_pre = len(wl.requests) * 0 + wl.n_prebuilt
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first_rid = None
    for r, p in zip(wl.requests, wl.plan):
        if not closed_loop:
            target = t0 + r["t"] / rate_scale
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                if target - now > 2e-4:
                    time.sleep(min(target - now - 1e-4, 5e-3))
        if p[0] == "build":
            keys, vals, seed, n, _ = wl.maps[p[1]]
            rid, mid = srv.submit_build(keys, vals, seed)
            map_ids.append(mid)
            outs.append(None)
        else:
            q = p[2]
            v = torch.empty(q.numel(), dtype=torch.int32, device=wl.device)
            f = torch.empty(q.numel(), dtype=torch.uint8, device=wl.device)
            rid = srv.submit_lookup(map_ids[p[1]], q, v, f)
            outs.append((v, f))
        if first_rid is None:
            first_rid = rid
    srv.wait_all()
    torch.cuda.synchronize()
    total = first_rid + len(wl.requests)
    sub, done, kind, status = srv.latencies(total)
    stats = srv.stats()
    srv.destroy()
    sub, done, kind, status = sub[first_rid:], done[first_rid:], kind[first_rid:], status[first_rid:]
    lat = done - sub
    res = {"requests": len(wl.requests), "status_ok": bool((status == 0).all()), "status": status.tolist(),
           "span_ms": float(done.max() - sub.min()), "stats": stats}
    for k, name in ((0, "build"), (1, "lookup")):
        sel = kind == k
        if sel.any():
            res[f"{name}_p50_ms"] = float(np.percentile(lat[sel], 50))
            res[f"{name}_p99_ms"] = float(np.percentile(lat[sel], 99))
            res[f"{name}_count"] = int(sel.sum())
            # p99 over the first and the last quarter of the stream (in submission order): a
            # queue that grows over the stream shows as a later p99 far above the earlier one
            ls = lat[sel]
            q = max(1, ls.size // 4)
            res[f"{name}_p99_first_quarter_ms"] = float(np.percentile(ls[:q], 99))
            res[f"{name}_p99_last_quarter_ms"] = float(np.percentile(ls[-q:], 99))
    # the slowest requests: what they were and when they arrived (ms after the first)
    worst = np.argsort(lat)[::-1][:5]
    sizes = [r["size"] for r in wl.requests]
    res["slowest"] = [{"kind": "build" if kind[i] == 0 else "lookup", "size": int(sizes[i]),
                       "latency_ms": round(float(lat[i]), 3), "submitted_at_ms": round(float(sub[i] - sub[0]), 3)}
                      for i in worst.tolist()]
    res["failed"] = int((status != 0).sum())
    res["failed_lookups"] = int(((status != 0) & (kind == 1)).sum())
    nq = sum(p[2].numel() for p in wl.plan if p[0] == "lookup")
    nk = sum(wl.maps[p[1]][3] for p in wl.plan if p[0] == "build")
    res["queries"] = int(nq)
    res["keys_built"] = int(nk)
    res["queries_per_s"] = nq / (res["span_ms"] * 1e-3)
    res["offered_rate_per_s"] = None if closed_loop else len(wl.requests) / (wl.requests[-1]["t"] / rate_scale)
    return res, outs


def check(wl: Workload, outs, status=None):
    """Every lookup's outputs against the exact expected answers.  With `status` (one entry
    per request, as the server reported it), lookups the server refused -- their map was
    evicted to make room -- are left out; every answered one must be exact."""
    import torch
    ok = True
    for i, (p, o) in enumerate(zip(wl.plan, outs)):
        if p[0] == "lookup":
            if status is not None and status[i] != 0:
                continue
            v, f = o
            ok &= bool(torch.equal(f, p[3])) and bool(torch.equal(v, p[4]))
    return ok


def stable(res, growth: float = 2.0, slack_ms: float = 1.0) -> bool:
    """Whether an open-loop replay kept up with its arrivals: the lookups' p99 over the last
    quarter of the stream stays within `growth` times (plus `slack_ms`) their p99 over the
    first quarter.  A queue that grows without bound makes later requests wait ever longer."""
    if "lookup_p99_last_quarter_ms" not in res or res["offered_rate_per_s"] is None:
        return False
    return res["lookup_p99_last_quarter_ms"] <= growth * res["lookup_p99_first_quarter_ms"] + slack_ms
