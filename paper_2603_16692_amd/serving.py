"""Continuous-batching request loop for KeySwitch calls of mixed parameter sets.

Requests (one polynomial d each, for one of several parameter sets) arrive at
arbitrary times. The scheduler keeps every set's evaluation key resident, holds
one FIFO queue per set, and whenever a stream slot is free and the HBM budget
allows, admits the oldest waiting set's queue head as a batch (up to that set's
batch limit), so that requests arriving while others run join the next batch
instead of waiting for a drain. Work on different streams overlaps on the
device. Completion is polled; each request's latency runs from its arrival to
the detection of its batch's completion. Batching never changes a result: the
KeySwitch of a batch item equals the KeySwitch of the item alone, bit for bit.

The device side is an Executor; GpuExecutor drives libks through torch streams,
and tests drive the same scheduler with a fake executor on the CPU.
"""
import collections
import dataclasses
import math
import random
import statistics
import time
from typing import Any, Dict, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    set_name: str
    payload: Any                  # d for this request (device tensor [ell][N] for the GPU executor)
    arrival: float = 0.0          # seconds on the scheduler clock
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Any = None
    batch_size: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Executor:
    """Device side of the loop: footprint of a batch, asynchronous launch, polling."""

    def footprint(self, set_name: str, batch: int) -> int:
        raise NotImplementedError

    def launch(self, set_name: str, requests: List[Request]) -> Any:
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> List[Any]:
        """Per-request results of a completed launch."""
        raise NotImplementedError

    def resident_bytes(self) -> int:
        return 0


class Scheduler:
    """Admission by HBM footprint, per-set FIFO batching, a fixed number of slots."""

    def __init__(self, executor: Executor, hbm_budget: int, max_batch: Dict[str, int], slots: int = 2,
                 clock=time.perf_counter, keep_results: bool = True):
        """keep_results=False drops each result once its request completes (a
        server hands it back to the client; holding every output of a long
        request stream would fill the device memory)."""
        if slots < 1:
            raise ValueError("need at least one slot")
        self.keep_results = keep_results
        self.ex = executor
        self.budget = hbm_budget
        self.max_batch = dict(max_batch)
        self.slots = slots
        self.clock = clock
        self.queues: Dict[str, collections.deque] = {k: collections.deque() for k in max_batch}
        self.inflight: List[tuple] = []   # (handle, set_name, requests, footprint)
        self.in_use = executor.resident_bytes()
        self.peak_in_use = self.in_use
        self.completed: List[Request] = []
        self.rejected: List[Request] = []
        self.launches = 0

    def submit(self, req: Request) -> bool:
        """Queue a request; a request whose single-item footprint can never fit is rejected."""
        if req.set_name not in self.queues:
            raise KeyError(req.set_name)
        if self.in_use_floor() + self.ex.footprint(req.set_name, 1) > self.budget:
            self.rejected.append(req)
            return False
        self.queues[req.set_name].append(req)
        return True

    def in_use_floor(self) -> int:
        return self.ex.resident_bytes()

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values()) + sum(len(r) for _, _, r, _ in self.inflight)

    def _poll(self) -> int:
        finished = 0
        still = []
        for h, name, reqs, fp in self.inflight:
            if self.ex.poll(h):
                now = self.clock()
                for r, res in zip(reqs, self.ex.finish(h)):
                    r.result, r.done = (res if self.keep_results else None), now
                    if not self.keep_results:
                        r.payload = None
                    self.completed.append(r)
                self.in_use -= fp
                finished += 1
            else:
                still.append((h, name, reqs, fp))
        self.inflight = still
        return finished

    def _admit(self) -> int:
        started = 0
        while len(self.inflight) < self.slots:
            heads = [(q[0].arrival, name) for name, q in self.queues.items() if q]
            if not heads:
                break
            _, name = min(heads)  # oldest waiting request first
            q = self.queues[name]
            b = min(len(q), self.max_batch[name])
            while b > 0 and self.in_use + self.ex.footprint(name, b) > self.budget:
                b -= 1
            if b == 0:
                break  # wait for memory to free up
            reqs = [q.popleft() for _ in range(b)]
            fp = self.ex.footprint(name, b)
            now = self.clock()
            for r in reqs:
                r.admitted, r.batch_size = now, b
            h = self.ex.launch(name, reqs)
            self.inflight.append((h, name, reqs, fp))
            self.in_use += fp
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.launches += 1
            started += 1
        return started

    def step(self) -> int:
        """Poll completions, then admit; returns how many launches changed state."""
        return self._poll() + self._admit()

    def run(self, requests: List[Request], offsets: List[float], idle_sleep: float = 0.0) -> List[Request]:
        """Submit requests[i] at start + offsets[i] (seconds) and serve until all are done.
        With keep_results=False each request also drops its payload once it
        completes."""
        order = sorted(range(len(requests)), key=lambda i: offsets[i])
        start = self.clock()
        nxt = 0
        while nxt < len(order) or self.pending():
            now = self.clock()
            while nxt < len(order) and start + offsets[order[nxt]] <= now:
                r = requests[order[nxt]]
                r.arrival = start + offsets[order[nxt]]
                self.submit(r)
                nxt += 1
            if self.step() == 0 and idle_sleep:
                time.sleep(idle_sleep)
        return self.completed


def poisson_offsets(n: int, rate: float, seed: int = 7) -> List[float]:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = random.Random(seed)
    t, out = 0.0, []
    for _ in range(n):
        t += rng.expovariate(rate)
        out.append(t)
    return out


def choose_sets(n: int, names: List[str], weights: List[float], seed: int = 7) -> List[str]:
    rng = random.Random(seed + 1)
    return rng.choices(names, weights=weights, k=n)


def latency_stats(done: List[Request]) -> Dict[str, float]:
    lat = sorted(r.latency for r in done if r.latency is not None)
    if not lat:
        return {"count": 0}

    def pct(p):
        return lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))]
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"count": len(lat), "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3,
            "mean_ms": statistics.mean(lat) * 1e3, "ks_per_s": len(lat) / span if span > 0 else float("nan")}


class GpuExecutor(Executor):
    """libks on the current device: one torch stream per slot, resident keys,
    and one workspace per (slot, set), allocated up front for the set's
    largest batch and reused by every launch on that slot (a launch then
    allocates only its stacked input and its output)."""

    def __init__(self, sets: Dict[str, Any], evks: Dict[str, Any], max_batch: Dict[str, int],
                 plans: Dict[str, Any] = None, slots: int = 2):
        import torch
        self.torch = torch
        self.sets = sets            # name -> KsParams
        self.evks = evks            # name -> resident device key
        self.plans = plans or {}
        self.max_batch = dict(max_batch)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free = list(range(slots))
        self._ws = {(si, name): G.workspace(self.max_batch[name], self.plans.get(name))
                    for si in range(slots) for name, G in sets.items()}

    def resident_bytes(self) -> int:
        keys = sum(int(e.numel()) * 8 for e in self.evks.values())
        return keys + sum(int(w.numel()) * 8 for w in self._ws.values())

    def footprint(self, set_name: str, batch: int) -> int:
        G = self.sets[set_name]
        return batch * (G.ell + 2 * G.ell) * G.n * 8  # d batch + out (the workspace is resident)

    def launch(self, set_name: str, requests: List[Request]):
        torch = self.torch
        G = self.sets[set_name]
        b = len(requests)
        if b > self.max_batch[set_name]:
            raise ValueError(f"{set_name}: batch {b} above the executor's limit {self.max_batch[set_name]}")
        si = self.free.pop()
        st = self.streams[si]
        plan = self.plans.get(set_name)
        st.wait_stream(torch.cuda.default_stream())  # the payloads were written there
        with torch.cuda.stream(st):
            d = torch.stack([r.payload for r in requests])
            out = torch.empty((b, 2, G.ell, G.n), dtype=torch.int64, device=d.device)
            G.keyswitch(d, self.evks[set_name], out, b, self._ws[(si, set_name)], plan, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, out, si, d)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> List[Any]:
        ev, out, si, d = handle
        self.free.append(si)
        return [out[i] for i in range(out.shape[0])]


def uniform_q_residues(moduli, count: int, n: int, gen, device="cuda"):
    """[count][len(moduli)][n] int64 residues, uniform modulo each modulus
    (all below 2^50 and above 2^49), drawn on the device from the torch
    generator `gen`: a 50-bit draw, replaced by a second 50-bit draw when it
    is not below the modulus, and by a third draw reduced modulo the modulus
    when that one is not either. Each modulus is within 2^-19 of 2^50 for the
    parameter sets here, so the last case has probability below 2^-38 per
    coefficient and the distribution is uniform up to that."""
    import torch
    if not all((1 << 49) < int(m) < (1 << 50) for m in moduli):
        raise ValueError("moduli must lie in (2^49, 2^50)")
    q = torch.tensor([int(m) for m in moduli], dtype=torch.int64, device=device)[None, :, None]
    shape = (count, len(moduli), n)
    r = torch.randint(0, 1 << 50, shape, generator=gen, device=device, dtype=torch.int64)
    r2 = torch.randint(0, 1 << 50, shape, generator=gen, device=device, dtype=torch.int64)
    r3 = torch.randint(0, 1 << 62, shape, generator=gen, device=device, dtype=torch.int64) % q
    return torch.where(r < q, r, torch.where(r2 < q, r2, r3))


# ------------------------------------------------------------------ benchmark

SERVE_SETS = {  # name: (dnum, log2 N, L, batch limit, share of requests)
    "d2-n13-l6": (2, 13, 6, 16, 0.4),
    "d2-n15-l10": (2, 15, 10, 32, 0.3),
    "d4-n16-l32": (4, 16, 32, 8, 0.2),
    "d8-n17-l56": (8, 17, 56, 2, 0.1),
}


def serve_benchmark(n_requests: int = 4000, loads=(0.5, 0.8), slots: int = 2, budget_gb: float = 96.0,
                    seed: int = 7) -> dict:
    """The mixed-parameter serving stream: Poisson arrivals, requests drawn
    40/30/20/10% from the four benchmark parameter sets, each with its own
    uniform random d (drawn on the device before the run: about 10 MB per
    request on average, 100 GB for 10 000 requests), resident keys, admission
    by HBM footprint, batching per set; against unbatched FIFO dispatch of
    the same trace on one stream. Both loads and both modes serve the same
    requests."""
    import numpy as np
    import torch

    from . import KsParams
    from synth import uniform_key

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")
    names = list(SERVE_SETS)
    shares = {k: v[4] for k, v in SERVE_SETS.items()}
    picks = choose_sets(n_requests, names, [shares[k] for k in names], seed=seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    sets, evks, payload = {}, {}, [None] * n_requests
    for name, (dn, ln, l, _, _) in SERVE_SETS.items():
        G = KsParams(dn, ln, l)
        sets[name] = G
        evks[name] = dev(uniform_key(G.moduli, G.n, G.ndig, seed=3))
        idx = [i for i in range(n_requests) if picks[i] == name]
        for c0 in range(0, len(idx), 64):  # 64 requests per draw bound the temporaries
            part = idx[c0:c0 + 64]
            d = uniform_q_residues(G.moduli[:l], len(part), G.n, gen)
            for j, i in enumerate(part):
                payload[i] = d[j]
    torch.cuda.synchronize()
    max_batch = {k: v[3] for k, v in SERVE_SETS.items()}
    # per-set plans from the shipped tuning table (the library default where none fits)
    from . import autotune
    table = autotune.shipped_cache()
    plans = {}
    for name, G in sets.items():
        p = autotune.plan_for(G, max_batch[name], table)
        if p is not None:
            plans[name] = p

    # batched service rate of each set alone (full batches back to back) -> capacity of the mix
    rate = {}
    for name, G in sets.items():
        b = max_batch[name]
        d = uniform_q_residues(G.moduli[:G.ell], b, G.n, gen)
        out = torch.empty((b, 2, G.ell, G.n), dtype=torch.int64, device="cuda")
        plan = plans.get(name)
        ws = G.workspace(b, plan)
        G.keyswitch(d, evks[name], out, b, ws, plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            G.keyswitch(d, evks[name], out, b, ws, plan)
        torch.cuda.synchronize()
        rate[name] = 5 * b / (time.perf_counter() - t0)
        del d, out, ws
    capacity = 1.0 / sum(shares[k] / rate[k] for k in sets)

    result = {"capacity_req_per_s": round(capacity, 1), "set_rates_ks_per_s": {k: round(v, 1) for k, v in rate.items()},
              "plans": {k: repr(v) for k, v in plans.items()},
              "requests": n_requests, "slots": slots, "runs": []}
    for load in loads:
        lam = load * capacity
        offs = poisson_offsets(n_requests, lam, seed=seed)
        row = {"load": load, "rate_req_per_s": round(lam, 1)}
        for mode, mb, sl in (("batched", max_batch, slots), ("unbatched", {k: 1 for k in names}, 1)):
            reqs = [Request(i, picks[i], payload[i]) for i in range(n_requests)]
            ex = GpuExecutor(sets, evks, mb, plans if mode == "batched" else {}, slots=sl)
            sched = Scheduler(ex, int(budget_gb * (1 << 30)), mb, slots=sl, keep_results=False)
            sched.run(reqs, offs)
            torch.cuda.synchronize()
            st = latency_stats(sched.completed)
            st["launches"] = sched.launches
            st["peak_hbm_gb"] = round(sched.peak_in_use / (1 << 30), 2)
            row[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            del ex, sched, reqs
            torch.cuda.empty_cache()
        result["runs"].append(row)
    return result


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="mixed-parameter KeySwitch serving benchmark")
    ap.add_argument("--requests", type=int, default=4000)
    ap.add_argument("--loads", default="0.5,0.8")
    ap.add_argument("--slots", type=int, default=2)
    args = ap.parse_args()
    out = serve_benchmark(args.requests, tuple(float(x) for x in args.loads.split(",")), args.slots)
    print(json.dumps(out))
