#!/usr/bin/env python3
"""Throughput of the CKKS hybrid KeySwitch on one MI355X.

One step = one batched KeySwitch (ModUp, KeyMult, ModDown for every
ciphertext of the batch) through libks, with inputs already resident in HBM.
Prints one JSON line: KeySwitch/s for the batch, the plain single-ciphertext
rate beside it, per-step latency percentiles, the roofline of the dominant
kernel (timed with HIP events inside the timed region) and the CPU oracle's
rate on a bounded sample of the same workload.

Inputs are synthetic (seeded SplitMix64): d uniform modulo each prime in NTT
form, and a uniform stand-in evaluation key of the real key's shape (a real
key is uniform modulo each prime as well).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# name: (dnum, log2 N, ell, batch, description)
WORKLOADS = {
    "d2-n13-l6": (2, 13, 6, 1, "plain KeySwitch (dnum,N,L)=(2,2^13,6)"),
    "d2-n15-l10": (2, 15, 10, 32, "batched KeySwitch (dnum,N,L)=(2,2^15,10), batch 32, shared evk"),
    "d4-n16-l32": (4, 16, 32, 8, "batched KeySwitch (dnum,N,L)=(4,2^16,32), batch 8, shared evk"),
    "d8-n17-l56": (8, 17, 56, 2, "deep-circuit KeySwitch (dnum,N,L)=(8,2^17,56), batch 2"),
}
HBM_PEAK_GBS = 8000.0
OP_METRIC = {"keyswitch": "KeySwitch/s", "hmul": "HMUL/s", "hrot": "HROT/s"}

# HBM bytes of one launch of the dominant kernel, from two rocprofv3 --pmc
# runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the same counter reads for a plain 1 GiB device copy
# (--copy-calibration): FETCH_SIZE reads half the copied bytes, WRITE_SIZE all
# of them. The figure holds only for the kernel sources it was measured on
# (sha256 below) and for the same workload and plan; otherwise "traffic" is null.
# The rocprofv3 summaries it comes from are under profiles/.
TRAFFIC = {"workload": "d4-n16-l32", "op": "keyswitch", "batch": 8, "plan": "Plan(DPOB, chunks=1, log_r=4, mfma)",
           "kernel": "moddown_blocks",
           "fetch_kib": 467292.4, "fetch_scale": 2.0, "write_kib": 262145.0, "write_scale": 1.0,
           "sources_sha256": "b3ff0a69815c593ee6725f96234da0a4136124b4acbe0f294b8cde32fe7a8e9d"}
TRAFFIC_SOURCES = ["paper_2603_16692_amd/csrc/ks_kernels.hip", "paper_2603_16692_amd/csrc/ks_device.hpp"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, op, batch, plan_repr, kernel):
    """HBM bytes per launch of `kernel` from the stored counters, or None."""
    t = TRAFFIC
    if (not t or t["workload"] != workload or t["op"] != op or t["batch"] != batch or t["plan"] != plan_repr
            or t["kernel"] != kernel):
        return None
    if t["sources_sha256"] != kernel_sources_sha256():
        return None
    return int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


def kernel_bytes(G, plan, batch, kind):
    """Algorithmic HBM bytes of all launches of `kind` in one step: each input
    a kernel needs read once, each output written once (the key once per
    batch). Digit-parallel plans run KeyMult for the P limbs only and fold the
    Q-limb KeyMult into ModDown's last block pass."""
    import paper_2603_16692_amd as ks
    W, N, B = 8, G.n, batch
    ell, nl, k, nd, a = G.ell, G.nl, G.k, G.ndig, G.alpha
    own = [len(range(j * a, min((j + 1) * a, ell))) for j in range(nd)]
    ext_q = sum(ell - o for o in own)   # raised Q limbs over all digits
    ext_p = nd * k                      # raised P limbs over all digits
    dp = plan.dataflow in (ks.DPOB, ks.DPOC)
    if kind == 0:    # inverse block pass of d
        return 2 * B * ell * N * W
    if kind == 1:    # ModUp columns: read the digits, write the raised limbs
        return B * ell * N * W + B * (ext_q + ext_p) * N * W
    if kind == 2:    # block pass + KeyMult
        if dp:       # P limbs: raised limbs in, key in once, acc_P out
            return B * ext_p * N * W + 2 * nd * k * N * W + 2 * B * k * N * W
        return B * (ext_q + ext_p) * N * W + B * ell * N * W + 2 * nd * nl * N * W + 2 * B * nl * N * W
    if kind == 3:    # ModDown columns: P limbs in, Q limbs out
        return 2 * B * k * N * W + 2 * B * ell * N * W
    if kind == 4:    # ModDown blocks: t2 in, out written; acc_Q in, or (DP) the Q KeyMult inputs
        if dp:
            return 2 * B * ell * N * W + B * ext_q * N * W + B * ell * N * W + 2 * nd * ell * N * W \
                + 2 * B * ell * N * W
        return 3 * 2 * B * ell * N * W
    if kind == 5:    # STAGED: forward block pass of every raised limb of ext, in place
        return 2 * B * (ext_q + ext_p) * N * W
    if kind == 6:    # STAGED: inverse block pass of the P limbs of acc into accp
        return 2 * 2 * B * k * N * W
    if kind == 7:    # STAGED: digit limbs of d copied into their ext slots
        return 2 * B * ell * N * W
    if kind == 8:    # STAGED: element-wise KeyMult over ext [B][dnum][ell+k][N]
        return B * nd * nl * N * W + 2 * nd * nl * N * W + 2 * B * nl * N * W
    return None


# FP64 modular products per second at the chip's vector rate: 256 CUs x 4 SIMDs
# x 16 lanes x 2.4 GHz = 39.3 T lane-operations/s, 6 FP64 operations per
# product (h = ab, l = fma(a, b, -h), h/q, rint, fma(-k, q, h), + l). The ALU
# roofline uses the rate the library's throughput probe measures in the same
# run (ks_modmul_rate); this derived figure is reported beside it.
MODMUL_DERIVED_T = 256 * 4 * 16 * 2.4e9 / 6 / 1e12


def ks_algorithmic_bytes(G, batch):
    """Algorithmic HBM bytes of one KeySwitch: d read once, out written once,
    the key read once per batch (d + out + evk / B)."""
    W, N, lv = 8, G.n, G.ell
    # the key rows of the (level's) digits and limbs: the whole key at the top level
    key_read = G.ndig * 2 * G.nl
    return lv * N * W + 2 * lv * N * W + key_read * N * W / batch


def kernel_modmuls(G, plan, batch, kind):
    """Algorithmic modular products of all launches of `kind` in one step (Q
    limbs, FP64): butterflies of its block passes (log M stages of N/2), key
    products and the final P^-1, or None for kinds not modelled."""
    import paper_2603_16692_amd as ks
    N, B, ell, nd = G.n, batch, G.ell, G.ndig
    log_m = G.log_n - plan.log_r
    if kind != 4:
        return None
    if plan.dataflow in (ks.DPOB, ks.DPOC):
        # per Q limb: both t2 components and the raised limb of every other digit
        return B * ell * ((nd + 1) * log_m * N // 2 + 2 * nd * N + 2 * N)
    return B * 2 * ell * (log_m * N // 2 + N)


# Descending level sequences of the level-sequence mode: a ciphertext that
# loses limbs as a circuit proceeds, switched at each level it passes.
LEVEL_SEQUENCES = {"d4-n16-l32": (32, 24, 16, 8), "d8-n17-l56": (56, 40, 24, 8), "d2-n15-l10": (10, 5)}


def level_sequence(args, dnum, log_n, ell, batch, desc):
    """One step = one batched KeySwitch at each level of a descending
    sequence (the same evaluation key throughout). Timed twice: each level
    under its own tuned plan (the shipped table; the library default where
    it has none) and every level under the top level's plan."""
    import numpy as np
    import torch

    import paper_2603_16692_amd as ks
    from paper_2603_16692_amd import autotune
    from synth import ciphertext_batch, uniform_key

    levels = (LEVEL_SEQUENCES[args.workload] if args.level_sequence == "default"
              else tuple(int(x) for x in args.level_sequence.split(",")))
    if any(not 1 <= lv <= ell for lv in levels) or list(levels) != sorted(levels, reverse=True):
        raise SystemExit(f"levels must descend within [1, {ell}]: {levels}")
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")
    top = ks.KsParams(dnum, log_n, ell)
    table = autotune.shipped_cache()
    top_plan = autotune.plan_for(top, batch, table) or top.default_plan(batch)
    evk = to_dev(uniform_key(top.moduli, top.n, top.ndig))
    runs = []
    for lv in levels:
        G = top.at_level(lv) if lv != ell else top
        tuned = autotune.cached_plan(G, batch, table)
        src = "shipped tuning table" if tuned is not None else "library default"
        tuned = tuned or G.default_plan(batch)
        d = to_dev(ciphertext_batch(G.moduli[:lv], G.n, batch))
        out = torch.empty((batch, 2, lv, G.n), dtype=torch.int64, device="cuda")
        runs.append({"level": lv, "G": G, "d": d, "out": out, "tuned": tuned, "source": src,
                     "ws": {"tuned": G.workspace(batch, tuned), "fixed": G.workspace(batch, top_plan)}})
    stream = torch.cuda.current_stream()
    result = {}
    for mode in ("tuned", "fixed"):
        def step():
            for r in runs:
                plan = r["tuned"] if mode == "tuned" else top_plan
                r["G"].keyswitch(r["d"], evk, r["out"], batch, r["ws"][mode], plan)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = ks.HipEvents(2 * len(runs) * args.steps)
        for i in range(args.steps):
            for j, r in enumerate(runs):
                plan = r["tuned"] if mode == "tuned" else top_plan
                ev.record(2 * (i * len(runs) + j), stream)
                r["G"].keyswitch(r["d"], evk, r["out"], batch, r["ws"][mode], plan)
                ev.record(2 * (i * len(runs) + j) + 1, stream)
        torch.cuda.synchronize()
        total = ev.elapsed_ms(0, 2 * len(runs) * args.steps - 1)
        per_level = [sum(ev.elapsed_ms(2 * (i * len(runs) + j), 2 * (i * len(runs) + j) + 1)
                         for i in range(args.steps)) / args.steps for j in range(len(runs))]
        result[mode] = {"ks_per_s": round(batch * len(runs) * args.steps / (total / 1e3), 2),
                        "ms_per_sequence": round(total / args.steps, 4),
                        "per_level_ms": {str(r["level"]): round(m, 4) for r, m in zip(runs, per_level)}}
    # every level's output is the same under both plans (each is bit-exact against the oracle in the tests)
    line = {
        "metric": "KeySwitch/s", "value": result["tuned"]["ks_per_s"], "unit": "KeySwitch/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": result["tuned"]["ms_per_sequence"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{desc}, one KeySwitch at each of the levels {list(levels)}",
                   "dnum": dnum, "N": top.n, "L": ell, "levels": list(levels), "batch": batch},
        "per_level_plans": {str(r["level"]): {"plan": repr(r["tuned"]), "source": r["source"]} for r in runs},
        "top_level_plan": repr(top_plan),
        "tuned": result["tuned"], "fixed_top_plan": result["fixed"],
        "gain_over_fixed": round(result["tuned"]["ks_per_s"] / result["fixed"]["ks_per_s"], 4),
    }
    print(json.dumps(line))


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d4-n16-l32", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=0, help="override the workload's batch size")
    ap.add_argument("--op", default="keyswitch", choices=["keyswitch", "hmul", "hrot"],
                    help="the timed operation: KeySwitch, or HMUL / HROT around it (same plan)")
    ap.add_argument("--level", type=int, default=0,
                    help="KeySwitch at this many Q limbs with the top-level key (default: the top level)")
    ap.add_argument("--plan", default="",
                    help="dataflow[,chunks[,log_r[,options]]], options mfma, split, hoist and tile=<items per pass> "
                         "joined by '+', e.g. DPOB or DSOC,2,3 or DPOB,1,4,mfma+split or DPOB,1,3,mfma+tile=8")
    ap.add_argument("--h2d", action="store_true",
                    help="with --op hmul: also time HMUL with its inputs copied from pinned host memory (overlapped)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default plan instead of tuning")
    ap.add_argument("--tune", action="store_true", help="tune even if a shipped tuned plan exists")
    ap.add_argument("--save-tuned", default="", help="merge the tuning winner into this JSON table")
    ap.add_argument("--tune-plans", type=int, default=0, help="candidate plans the tuner times (0 = all)")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay measurement")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain single-ciphertext measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--level-sequence", default="",
                    help="comma-separated descending levels (or 'default'): time one KeySwitch of the batch at "
                         "each level in turn, with per-level tuned plans and with the top level's plan")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported: the KeySwitch path is "
              "single-GPU (batch sharding across GPUs, which needs no communication, is not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_16692_amd as ks
    from synth import ciphertext_batch, uniform_key

    if args.copy_calibration:
        n = 1 << 27  # 2^27 int64 words = 1 GiB
        src = torch.ones(n, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        ev = ks.HipEvents(2)
        for _ in range(2):
            dst.copy_(src)
        ev.record(0)
        dst.copy_(src)
        ev.record(1)
        torch.cuda.synchronize()
        ms = ev.elapsed_ms(0, 1)
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "ms": round(ms, 4),
                          "GBs": round(2 * n * 8 / (ms / 1e3) / 1e9, 1)}))
        return

    dnum, log_n, ell, batch, desc = WORKLOADS[args.workload]
    if args.batch:
        batch = args.batch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.level_sequence:
        level_sequence(args, dnum, log_n, ell, batch, desc)
        return
    top = ks.KsParams(dnum, log_n, ell)
    G = top.at_level(args.level) if args.level else top
    if args.level:
        desc += f" at level {args.level}"

    plan = None
    if args.plan:
        parts = args.plan.split(",")
        df = {"DSOB": ks.DSOB, "DPOB": ks.DPOB, "DSOC": ks.DSOC, "DPOC": ks.DPOC, "STAGED": ks.STAGED}[parts[0]]
        chunks = int(parts[1]) if len(parts) > 1 else 1
        log_r = int(parts[2]) if len(parts) > 2 else -1
        opts = parts[3].split("+") if len(parts) > 3 else []
        tile = next((int(o[5:]) for o in opts if o.startswith("tile=")), 0)
        plan = ks.make_plan(df, chunks, log_r, "mfma" in opts, "split" in opts, tile, "hoist" in opts)

    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")
    lv = G.ell
    d = to_dev(ciphertext_batch(G.moduli[:lv], G.n, batch))
    evk = to_dev(uniform_key(top.moduli, top.n, top.ndig))  # the top-level key
    out = torch.empty((batch, 2, lv, G.n), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    tuning = None
    if plan is None and not args.tune and not args.no_tune:
        # the plan an earlier tuning run on this hardware chose, if shipped
        from paper_2603_16692_amd import autotune
        plan = autotune.cached_plan(G, batch, autotune.shipped_cache())
        if plan is not None:
            tuning = {"source": "shipped tuning table", "plan": repr(plan)}
    if plan is None and args.no_tune:
        plan = G.default_plan(batch)
    elif plan is None:
        # per-parameter dataflow choice by measurement (untimed setup)
        from paper_2603_16692_amd import autotune
        cands = autotune.prior_order(G, batch, autotune.candidate_plans(G, batch))
        table = autotune.load_cache(args.save_tuned) if args.save_tuned else {}
        plan, results = autotune.tune(G, d, evk, batch, plans=cands[:args.tune_plans] if args.tune_plans else cands,
                                      reps=3, trials=2, cache=table)
        if args.save_tuned:
            autotune.save_cache(table, args.save_tuned)
        ranked = sorted(results, key=lambda r: r["ms"])
        tuning = {"source": "tuned in this run", "plans_tried": len(results), "best": ranked[0]["name"],
                  "best_ms": round(ranked[0]["ms"], 4), "worst": ranked[-1]["name"],
                  "worst_ms": round(ranked[-1]["ms"], 4),
                  "default_ms": round(next((r["ms"] for r in results
                                            if tuple(r["plan"]) == G.default_plan(batch).key()), float("nan")), 4)}
    ws = G.workspace(batch, plan)
    if args.op == "keyswitch":
        step = lambda: G.keyswitch(d, evk, out, batch, ws, plan)
    else:
        # a second operand of the same shape; the key plays the relinearisation or rotation key
        ews = G.eval_workspace(batch, plan)
        ct = to_dev(ciphertext_batch(G.moduli[:lv], G.n, 2 * batch, seed_base=2000)).view(batch, 2, lv, G.n)
        ct2 = to_dev(ciphertext_batch(G.moduli[:lv], G.n, 2 * batch, seed_base=3000)).view(batch, 2, lv, G.n)
        if args.op == "hmul":
            step = lambda: G.hmul(ct, ct2, evk, out, batch, ews, plan)
        else:
            step = lambda: G.hrot(ct, 5, evk, out, batch, ews, plan)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-kernel breakdown of one step (untimed) -> the dominant kernel kind
    ev = ks.HipEvents(2 * 256)
    ks.trace_begin(ev)
    step()
    kinds = ks.trace_end()
    torch.cuda.synchronize()
    per_kind = {}
    for i, kd in enumerate(kinds):
        per_kind[kd] = per_kind.get(kd, 0.0) + ev.elapsed_ms(2 * i, 2 * i + 1)
    dominant = max(per_kind, key=per_kind.get)

    # timed region: K steps between two HIP events on the stream the kernels
    # run on; every launch of the dominant kernel inside it is bracketed by
    # HIP events as well
    run_ev = ks.HipEvents(2)
    per_step = sum(1 for k in kinds if k == dominant)
    kev = ks.HipEvents(2 * args.steps * per_step)
    torch.cuda.synchronize()
    ks.trace_begin(kev, 1 << dominant)
    wall0 = time.perf_counter()
    run_ev.record(0, stream)
    for i in range(args.steps):
        step()
    run_ev.record(1, stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    dom_kinds = ks.trace_end(kev.count // 2)
    total_ms = run_ev.elapsed_ms(0, 1)
    dom_ms = [kev.elapsed_ms(2 * i, 2 * i + 1) for i in range(len(dom_kinds))]
    ms_per_step = total_ms / args.steps
    value = batch * args.steps / (total_ms / 1e3)

    # per-step latency in a pass of its own (an event after every step costs
    # the host and the queue a little, which the timed region should not carry)
    step_ev = ks.HipEvents(args.steps + 1)
    step_ev.record(0, stream)
    for i in range(args.steps):
        step()
        step_ev.record(i + 1, stream)
    torch.cuda.synchronize()
    step_ms = [step_ev.elapsed_ms(i, i + 1) for i in range(args.steps)]

    # plain single-ciphertext path on the same parameters (the shipped
    # one-ciphertext plan of this set if there is one, else the default plan)
    plain = plain_plan = None
    if batch > 1 and not args.no_plain and args.op == "keyswitch":
        from paper_2603_16692_amd import autotune
        p1 = autotune.cached_plan(G, 1, autotune.shipped_cache())
        plain_plan = repr(p1) if p1 is not None else "default " + repr(G.default_plan(1))
        d1 = d[:1].contiguous()
        out1 = out[:1].contiguous()
        ws1 = G.workspace(1, p1)
        for _ in range(3):
            G.keyswitch(d1, evk, out1, 1, ws1, p1)
        pe = ks.HipEvents(2)
        reps = max(10, args.steps)
        pe.record(0, stream)
        for _ in range(reps):
            G.keyswitch(d1, evk, out1, 1, ws1, p1)
        pe.record(1, stream)
        torch.cuda.synchronize()
        plain = reps / (pe.elapsed_ms(0, 1) / 1e3)

    # the same step replayed from a captured HIP graph
    graph_rate = None
    if not args.no_graph and args.op == "keyswitch":
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        with torch.cuda.stream(gs):
            g = G.graph(d, evk, out, batch, ws, plan, stream=gs)
            for _ in range(2):
                g.launch(gs)
            ge = ks.HipEvents(2)
            ge.record(0, gs)
            for _ in range(args.steps):
                g.launch(gs)
            ge.record(1, gs)
        torch.cuda.synchronize()
        graph_rate = batch * args.steps / (ge.elapsed_ms(0, 1) / 1e3)
        del g

    # HMUL with its inputs copied from pinned host memory inside the timed
    # region (the paper's timed operation includes this copy): the copy of
    # batch i + 1 runs on a second stream while batch i computes, into two
    # device buffer sets
    h2d = None
    if args.h2d and args.op == "hmul":
        host = [t.cpu().pin_memory() for t in (ct, ct2)]
        bufs = [[torch.empty_like(ct), torch.empty_like(ct2)] for _ in range(2)]
        cs = torch.cuda.Stream()
        copied = [torch.cuda.Event() for _ in range(2)]
        used = [torch.cuda.Event() for _ in range(2)]
        nbytes_in = sum(t.numel() * 8 for t in host)

        def h2d_steps(n, compute=True):
            for i in range(n):
                k = i % 2
                with torch.cuda.stream(cs):
                    if i >= 2:
                        cs.wait_event(used[k])  # the compute that read this buffer set is done
                    for dst, src in zip(bufs[k], host):
                        dst.copy_(src, non_blocking=True)
                    copied[k].record(cs)
                stream.wait_event(copied[k])
                if compute:
                    G.hmul(bufs[k][0], bufs[k][1], evk, out, batch, ews, plan)
                used[k].record(stream)

        reps = max(10, args.steps // 4)
        h2d_steps(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h2d_steps(reps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        h2d_steps(reps, compute=False)
        torch.cuda.synchronize()
        dc = time.perf_counter() - t0
        h2d = {"value": round(batch * reps / dt, 2), "unit": "HMUL/s", "steps": reps,
               "input_bytes_per_step": nbytes_in, "copy_only_GBs": round(nbytes_in * reps / dc / 1e9, 1)}
        del bufs, host

    # Roofline of the dominant kernel. "achieved" counts the KeySwitch's
    # algorithmic bytes (d + out + evk / B per KeySwitch) for the KeySwitches
    # one launch completes (batch / launches per step), over the average
    # launch time. The bytes the kernel itself must stage (its inputs read
    # once, its outputs written once, intermediates included) are reported
    # beside it as staged_bytes_per_launch, the HBM bytes the counters saw as
    # traffic, and traffic / algorithmic bytes as wasted_traffic.
    dom_avg_ms = sum(dom_ms) / len(dom_ms)
    ks_bytes = ks_algorithmic_bytes(G, batch)
    alg_per_launch = ks_bytes * batch / per_step
    achieved = alg_per_launch / (dom_avg_ms / 1e3) / 1e9
    staged = kernel_bytes(G, plan, batch, dominant)
    traffic = (measured_traffic(args.workload, args.op, batch, repr(plan), ks.KIND_NAMES[dominant])
               if not args.level else None)
    step_GBs = ks_bytes * value / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ks.KIND_NAMES[dominant], "kernel_avg_ms": round(dom_avg_ms, 4),
                "launches_per_step": per_step, "keyswitches_per_launch": batch / per_step,
                "algorithmic_bytes_per_keyswitch": int(ks_bytes),
                "algorithmic_bytes_per_launch": int(alg_per_launch),
                "staged_bytes_per_launch": int(staged / per_step) if staged is not None else None,
                "step_GBs": round(step_GBs, 1), "step_frac": round(step_GBs / HBM_PEAK_GBS, 4)}
    if staged is not None:
        roofline["staged_frac"] = round(staged / per_step / (dom_avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if traffic:
        # bytes that left L2 (MALL hits included) and came back, per second of the kernel
        roofline["measured_GBs"] = round(traffic / (dom_avg_ms / 1e3) / 1e9, 1)
        roofline["measured_frac"] = round(roofline["measured_GBs"] / HBM_PEAK_GBS, 4)
        roofline["wasted_traffic"] = round(traffic / alg_per_launch, 2)

    # the practical streaming ceiling: the library's copy probe at the access
    # widths the kernels use (8 and 16 bytes per lane), cached and
    # non-temporal stores, over 1 GiB read + 1 GiB written
    copy = {f"{8 * (k + 1)}B{'_nt' if nt else ''}": round(ks.copy_rate(k, nt) / 1e9, 1)
            for k in (0, 1) for nt in (False, True)}
    roofline["copy_ceiling_GBs"] = copy
    roofline["frac_of_copy_ceiling"] = round(achieved / max(copy.values()), 4)

    roofline_alu = None
    nmm = kernel_modmuls(G, plan, batch, dominant) if args.op == "keyswitch" else None
    if nmm is not None:
        peaks = {name: G.modmul_rate(kind) / 1e12 for kind, name in ((0, "fp64"), (1, "shoup"), (2, "montgomery"))}
        rate = nmm / per_step / (dom_avg_ms / 1e3) / 1e12
        roofline_alu = {"bound": "alu", "achieved": round(rate, 3), "peak": round(peaks["fp64"], 3),
                        "unit": "T modmul/s", "frac": round(rate / peaks["fp64"], 4), "kernel": ks.KIND_NAMES[dominant],
                        "modmuls_per_launch": int(nmm / per_step),
                        "peak_source": "ks_modmul_rate (FP64 products modulo a Q prime), measured in this run",
                        "measured_peaks_T": {k: round(v, 3) for k, v in peaks.items()},
                        "derived_fp64_peak_T": round(MODMUL_DERIVED_T, 3)}

    cpu = None
    if not args.no_cpu_baseline and args.op == "keyswitch":
        import oracle
        top_p = oracle.Params(dnum, log_n, ell)
        P = top_p.at_level(lv)
        dh = ciphertext_batch(P.q, P.n, 1)
        kh = uniform_key(top_p.moduli, P.n, top_p.ndig)
        n_done, t_start = 0, time.perf_counter()
        while True:
            oracle.keyswitch(P, dh, kh, 1)
            n_done += 1
            el = time.perf_counter() - t_start
            if el >= args.cpu_seconds or el / n_done * (n_done + 1) > 3 * args.cpu_seconds:
                break
        cores = oracle.max_threads()
        cpu = {"value": round(n_done / el, 4), "unit": "KeySwitch/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{n_done} single-ciphertext KeySwitch(es) of the same parameter set, {el:.1f} s"}
        # the same oracle on one thread, on a sample of about a third of the time
        oracle.set_threads(1)
        try:
            n1, t_start = 0, time.perf_counter()
            while True:
                oracle.keyswitch(P, dh, kh, 1)
                n1 += 1
                el1 = time.perf_counter() - t_start
                if el1 >= args.cpu_seconds / 3 or el1 / n1 * (n1 + 1) > args.cpu_seconds:
                    break
        finally:
            oracle.set_threads(cores)
        cpu["single_thread"] = {"value": round(n1 / el1, 4), "unit": "KeySwitch/s", "cores": 1,
                                "sample": f"{n1} single-ciphertext KeySwitch(es), {el1:.1f} s"}

    line = {
        "metric": OP_METRIC[args.op], "value": round(value, 2), "unit": OP_METRIC[args.op], "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "dnum": dnum, "N": G.n, "L": ell, "level": lv, "k": G.k, "batch": batch,
                   "plan": repr(plan), "launches_per_step": len(kinds)},
        "plain_single_ks_per_s": round(plain, 2) if plain else None,
        "plain_single_plan": plain_plan,
        "graph_ks_per_s": round(graph_rate, 2) if graph_rate else None,
        "h2d_inclusive": h2d,
        "autotune": tuning,
        "latency_ms": {"p50": round(percentile(step_ms, 50), 4), "p99": round(percentile(step_ms, 99), 4)},
        "ks_algorithmic_GBs": round(step_GBs, 1),
        "breakdown_ms": {ks.KIND_NAMES[k]: round(v, 4) for k, v in sorted(per_kind.items())},
        "wall_s": round(wall1 - wall0, 4),
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
