"""GPU tests of the runtime around the kernels: HIP-graph replay, the
autotuner's plan choice, and the continuous-batching loop. Every result is
compared bit for bit with an eager call, a batch-1 call, or the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import ciphertext_batch

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
                                                                 (2, 15, 10, 5, 1, 3, 2)])
def test_graph_replay_matches_eager(ks, dnum, log_n, ell, batch, df, flags, tile):
    """Replays of a captured KeySwitch equal eager calls; flags 2 (a batch
    split over two streams) captures a fork and a join of the second stream,
    a batch tile several passes over one workspace."""
    G = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    _, _, evk = oracle.keygen(P, h=64)
    plan = ks.make_plan(df, 2 if df in (ks.DSOC, ks.DPOC) else 1, 3 if flags & 1 else -1,
                        mfma=bool(flags & 1), split=bool(flags & 2), tile=tile)
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


def test_serving_results_equal_alone(ks):
    from paper_2603_16692_amd.serving import GpuExecutor, Request, Scheduler, choose_sets, poisson_offsets
    specs = {"small": (2, 13, 6), "mid": (2, 15, 10), "odd": (3, 12, 7)}
    sets, evks, ps = {}, {}, {}
    for name, (dn, ln, l) in specs.items():
        sets[name] = ks.KsParams(dn, ln, l)
        ps[name] = oracle.Params(dn, ln, l)
        evks[name] = dev(oracle.keygen(ps[name], h=64)[2])
    n = 60
    names = choose_sets(n, list(specs), [0.4, 0.4, 0.2], seed=11)
    offs = poisson_offsets(n, 4000.0, seed=11)
    reqs = []
    for i in range(n):
        P = ps[names[i]]
        reqs.append(Request(i, names[i], dev(ciphertext_batch(P.q, P.n, 1, seed_base=5000 + i)[0])))
    torch.cuda.synchronize()
    ex = GpuExecutor(sets, evks, slots=2)
    sched = Scheduler(ex, hbm_budget=8 << 30, max_batch={"small": 4, "mid": 8, "odd": 3}, slots=2)
    done = sched.run(reqs, offs)
    torch.cuda.synchronize()
    assert len(done) == n
    assert max(r.batch_size for r in done) > 1, "no request was batched"
    for r in done:
        G = sets[r.set_name]
        out = empty((1, 2, G.ell, G.n))
        G.keyswitch(r.payload[None].contiguous(), evks[r.set_name], out, 1, G.workspace(1))
        assert first_mismatch(host(r.result[None].contiguous()), host(out)) is None, f"request {r.rid}"
    # a sample against the oracle
    for r in done[:3]:
        P = ps[r.set_name]
        d = host(r.payload[None].contiguous())
        ref = oracle.keyswitch(P, d, host(evks[r.set_name]).reshape(P.ndig, 2, P.nl, P.n), 1)
        assert first_mismatch(host(r.result[None].contiguous()), ref) is None
