"""GPU tests of the runtime around the kernels: HIP-graph replay, the
autotuner's plan choice, and the continuous-batching loop. Every result is
compared bit for bit with an eager call, a batch-1 call, or the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from synth import ciphertext_batch, uniform_key

from gpu_util import dev, empty, first_mismatch, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_16692_amd as k
    return k


@pytest.mark.parametrize("dnum,log_n,ell,batch,df,flags,tile", [(2, 15, 10, 4, 1, 0, 0), (4, 16, 32, 2, 1, 0, 0),
                                                                 (2, 13, 6, 1, 0, 0, 0), (3, 12, 7, 3, 3, 0, 0),
                                                                 (2, 15, 10, 4, 1, 3, 0), (3, 12, 7, 3, 4, 2, 0),
                                                                 (2, 15, 10, 5, 1, 3, 2), (2, 13, 6, 1, 1, 4, 0),
                                                                 (3, 12, 7, 3, 1, 7, 0)])
def test_graph_replay_matches_eager(ks, dnum, log_n, ell, batch, df, flags, tile):
    """Replays of a captured KeySwitch equal eager calls; flags 2 (a batch
    split over two streams) captures a fork and a join of the second stream,
    a batch tile several passes over one workspace."""
    G = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    _, _, evk = oracle.keygen(P, h=64)
    plan = ks.make_plan(df, 2 if df in (ks.DSOC, ks.DPOC) else 1, 3 if flags & 1 else -1,
                        mfma=bool(flags & 1), split=bool(flags & 2), tile=tile, hoist=bool(flags & 4))
    ee = dev(evk)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = empty((batch, ell, P.n))
        out = empty((batch, 2, ell, P.n))
        ws = G.workspace(batch, plan)
        d.copy_(dev(ciphertext_batch(P.q, P.n, batch, seed_base=50)))
        g = G.graph(d, ee, out, batch, ws, plan, stream=s)
    s.synchronize()
    other = ks.KsParams(2, 13, 6)
    _, _, evk_o = oracle.keygen(oracle.Params(2, 13, 6), h=64)
    for rep in range(4):
        inputs = ciphertext_batch(P.q, P.n, batch, seed_base=100 + 10 * rep)
        with torch.cuda.stream(s):
            d.copy_(dev(inputs))
            g.launch(s)
        s.synchronize()
        got = host(out).copy()
        # eager work of the program between replays
        eo = empty((1, 2, 6, 1 << 13))
        other.keyswitch(dev(ciphertext_batch(oracle.Params(2, 13, 6).q, 1 << 13, 1)), dev(evk_o), eo, 1,
                        other.workspace(1))
        torch.cuda.synchronize()
        e_out = empty((batch, 2, ell, P.n))
        G.keyswitch(dev(inputs), ee, e_out, batch, G.workspace(batch, plan), plan)
        ref = host(e_out)
        assert first_mismatch(got, ref) is None, f"replay {rep}"
        if rep == 0:
            assert first_mismatch(ref, oracle.keyswitch(P, inputs, evk, batch)) is None


def test_autotuner_keeps_only_bit_exact_plans(ks):
    from paper_2603_16692_amd import autotune
    G = ks.KsParams(3, 14, 9)
    P = oracle.Params(3, 14, 9)
    _, _, evk = oracle.keygen(P, h=64)
    batch = 3
    d = ciphertext_batch(P.q, P.n, batch)
    plans = autotune.prior_order(G, batch, autotune.candidate_plans(G, batch))
    assert len(plans) >= 20
    cache = {}
    best, results = autotune.tune(G, dev(d), dev(evk), batch, plans=plans[:12], reps=2, trials=1, cache=cache)
    assert all(r["bit_exact"] for r in results)
    assert autotune.cached_plan(G, batch, cache).key() == best.key()
    out = empty((batch, 2, P.ell, P.n))
    G.keyswitch(dev(d), dev(evk), out, batch, G.workspace(batch, best), best)
    assert first_mismatch(host(out), oracle.keyswitch(P, d, evk, batch)) is None


def _serve_and_check(ks, specs, weights, max_batch, n, rate, seed, oracle_checks, plans=None):
    """Serve n requests of mixed sets through the continuous-batching loop;
    every result must equal the KeySwitch of its request alone, and a few
    must equal the oracle's."""
    from paper_2603_16692_amd.serving import GpuExecutor, Request, Scheduler, choose_sets, poisson_offsets
    sets, evks, ps, hevk = {}, {}, {}, {}
    for name, (dn, ln, l) in specs.items():
        sets[name] = ks.KsParams(dn, ln, l)
        ps[name] = oracle.Params(dn, ln, l)
        # the oracle's key for the small sets; a uniform key of the same shape for the large ones
        hevk[name] = (oracle.keygen(ps[name], h=64)[2] if ln <= 15 else
                      uniform_key(ps[name].moduli, ps[name].n, ps[name].ndig))
        evks[name] = dev(hevk[name])
    names = choose_sets(n, list(specs), weights, seed=seed)
    offs = poisson_offsets(n, rate, seed=seed)
    reqs = []
    for i in range(n):
        P = ps[names[i]]
        reqs.append(Request(i, names[i], dev(ciphertext_batch(P.q, P.n, 1, seed_base=5000 + i)[0])))
    torch.cuda.synchronize()
    ex = GpuExecutor(sets, evks, max_batch, plans, slots=2)
    sched = Scheduler(ex, hbm_budget=64 << 30, max_batch=max_batch, slots=2)
    done = sched.run(reqs, offs)
    torch.cuda.synchronize()
    assert len(done) == n
    assert max(r.batch_size for r in done) > 1, "no request was batched"
    for r in done:
        G = sets[r.set_name]
        out = empty((1, 2, G.ell, G.n))
        G.keyswitch(r.payload[None].contiguous(), evks[r.set_name], out, 1, G.workspace(1))
        assert first_mismatch(host(r.result[None].contiguous()), host(out)) is None, f"request {r.rid}"
    checked = set()
    for r in done:  # against the oracle: the first request of each named set
        if r.set_name in oracle_checks and r.set_name not in checked:
            checked.add(r.set_name)
            P = ps[r.set_name]
            d = host(r.payload[None].contiguous())
            ref = oracle.keyswitch(P, d, hevk[r.set_name], 1)
            assert first_mismatch(host(r.result[None].contiguous()), ref) is None, r.set_name
    assert checked == set(oracle_checks)
    return done


def test_serving_results_equal_alone(ks):
    specs = {"small": (2, 13, 6), "mid": (2, 15, 10), "odd": (3, 12, 7)}
    _serve_and_check(ks, specs, [0.4, 0.4, 0.2], {"small": 4, "mid": 8, "odd": 3}, 60, 4000.0, 11,
                     ("small", "mid", "odd"))


def test_serving_mix_of_the_four_benchmark_sets(ks):
    # the serving stream's mix: 40/30/20/10% of (2,2^13,6), (2,2^15,10),
    # (4,2^16,32) and (8,2^17,56), each set under its shipped plan, batches of
    # up to 16/32/8/2; results equal those of each request alone
    from paper_2603_16692_amd import autotune
    specs = {"d2-n13-l6": (2, 13, 6), "d2-n15-l10": (2, 15, 10), "d4-n16-l32": (4, 16, 32),
             "d8-n17-l56": (8, 17, 56)}
    max_batch = {"d2-n13-l6": 16, "d2-n15-l10": 32, "d4-n16-l32": 8, "d8-n17-l56": 2}
    probe = {k: ks.KsParams(*v) for k, v in specs.items()}
    plans = {k: autotune.plan_for(G, max_batch[k], autotune.shipped_cache()) for k, G in probe.items()}
    del probe
    done = _serve_and_check(ks, specs, [0.4, 0.3, 0.2, 0.1], max_batch, 80, 6000.0, 13,
                            ("d2-n13-l6", "d4-n16-l32"), plans)
    big = [r for r in done if r.set_name in ("d4-n16-l32", "d8-n17-l56")]
    assert big and any(r.batch_size > 1 for r in big), "no large-set request was batched"


def test_probes_compute_what_they_time(ks):
    # ks_modmul_rate (kind 0, FP64 products modulo the first Q prime): thread
    # t's word is the sum over its chains c of (8t + c + 1) * w^iters mod q
    G = ks.KsParams(2, 13, 6)
    q = G.moduli[0]
    w = q // 3 + 1
    blocks, iters = 2, 7
    sink = torch.zeros(blocks * 256, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert ks.raw_call("ks_modmul_rate", G._h, 0, blocks, iters, ctypes.c_void_p(sink.data_ptr()), stream) == 0
    chains = ks.raw_call("ks_modmul_chains")
    got = host(sink)
    wp = pow(w, iters, q)
    for t in (0, 1, 255, 300, blocks * 256 - 1):
        want = sum((chains * t + c + 1) * wp for c in range(chains)) % q
        assert int(got[t]) == want, t
    for kind in (1, 2):  # the integer products run and write every thread's word
        sink.fill_(0)
        assert ks.raw_call("ks_modmul_rate", G._h, kind, blocks, iters, ctypes.c_void_p(sink.data_ptr()), stream) == 0
        assert int(torch.count_nonzero(sink)) == blocks * 256
    assert ks.raw_call("ks_modmul_rate", G._h, 3, blocks, iters, ctypes.c_void_p(sink.data_ptr()), stream) == ks.KS_EINVAL
    # ks_copy_rate copies every word, with 8- and 16-byte accesses, cached and non-temporal
    src = torch.arange(1, 4097, dtype=torch.int64, device="cuda")
    for kind in (0, 1):
        for nt in (0, 1):
            dst = torch.zeros_like(src)
            rc = ks.raw_call("ks_copy_rate", kind, nt, 3, ctypes.c_void_p(src.data_ptr()),
                             ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(4096), stream)
            assert rc == 0
            assert torch.equal(dst, src), (kind, nt)
    assert ks.raw_call("ks_copy_rate", 1, 0, 3, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                       ctypes.c_size_t(4095), stream) == ks.KS_EINVAL
    torch.cuda.synchronize()
