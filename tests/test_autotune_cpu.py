"""Host logic of the autotuner: candidate enumeration, the footprint prior,
and the tuning table lookups (no GPU: a stand-in parameter object that
accepts plans the way libks does)."""
import paper_2603_16692_amd as ks
from paper_2603_16692_amd import autotune


class FakeParams:
    """Accepts a plan when libks would: NTT split within the compiled range,
    chunks within ell, the MFMA BConv only up to 32 rows per column and
    16 sources, with its packed digits within the 160 KB of LDS."""

    def __init__(self, dnum, log_n, ell, top_ell=None):
        self.dnum, self.log_n, self.ell = dnum, log_n, ell
        self.n = 1 << log_n
        self.alpha = -(-(top_ell or ell) // dnum)
        self.k = self.alpha
        self.ndig = -(-ell // self.alpha)
        self.nl = ell + self.k

    def workspace_bytes(self, batch, plan=None):
        log_m = self.log_n - plan.log_r
        if plan.log_r > 5 or log_m < 3 or log_m > 14:
            raise ks.KsError(ks.KS_EUNSUP, "split")
        nm = -(-max(self.alpha, self.k) // 4)
        if (plan.flags & ks.PLAN_MFMA_BCONV) and (nm > 4 or nm * (32 << plan.log_r) * 64 > 160 * 1024):
            raise ks.KsError(ks.KS_EUNSUP, "mfma")
        if plan.dataflow in (ks.DSOC, ks.DPOC) and not 1 <= plan.chunks <= min(64, self.ell):
            raise ks.KsError(ks.KS_EUNSUP, "chunks")
        per_pass = min(batch, plan.batch_tile) if plan.batch_tile else batch
        return per_pass * self.nl * self.n * 8

    def launch_count(self, batch, plan):
        return {ks.DPOB: 5, ks.STAGED: 8}.get(plan.dataflow, 5 * plan.chunks * self.ndig)


def test_candidates_cover_both_bconv_variants():
    P = FakeParams(4, 16, 32)
    plans = autotune.candidate_plans(P, 8)
    keys = {p.key() for p in plans}
    assert (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV, 0) in keys and (ks.DPOB, 1, 4, 0, 0) in keys
    assert (ks.DPOB, 1, 5, 0, 0) in keys and (ks.DPOB, 1, 5, ks.PLAN_MFMA_BCONV, 0) in keys
    # 32 rows of 12-prime digits exceed the LDS of the MFMA BConv
    wide = {p.key() for p in autotune.candidate_plans(FakeParams(1, 12, 12), 1)}
    assert (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV, 0) in wide and (ks.DPOB, 1, 5, ks.PLAN_MFMA_BCONV, 0) not in wide
    assert all(p.log_r >= 2 for p in plans)  # blocks of at most 2^14
    assert len(keys) == len(plans)
    # the batch split over two streams is a candidate only when there are two items
    split = ks.PLAN_SPLIT_STREAMS
    assert (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV | split, 0) in keys
    assert not any(p.flags & split for p in autotune.candidate_plans(P, 1))
    # the hoisted forward pass is a DPOB candidate only
    hoist = ks.PLAN_HOIST_FWD
    assert (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV | hoist, 0) in keys
    assert all(p.dataflow == ks.DPOB for p in plans if p.flags & hoist)
    # batch tiles of B/2 and B/4 for the digit-parallel plans, none below a batch of 4
    assert (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV, 4) in keys and (ks.STAGED, 1, 4, 0, 2) in keys
    assert not any(p.batch_tile and p.dataflow not in (ks.DPOB, ks.STAGED) for p in plans)
    assert not any(p.batch_tile for p in autotune.candidate_plans(P, 3))


def test_footprint_model_and_prior():
    # Table III: DS holds N*L words, DP dnum times that, OC divides by the chunks
    assert autotune.footprint_bytes(2, 1 << 15, 10, ks.DPOB) == 2 * (1 << 15) * 10 * 8
    assert autotune.footprint_bytes(2, 1 << 15, 10, ks.DSOB) == (1 << 15) * 10 * 8
    assert autotune.footprint_bytes(4, 1 << 16, 32, ks.DPOC, chunks=4, batch=8) == 4 * (1 << 16) * 32 * 8 * 8 // 4
    P = FakeParams(2, 15, 10)
    order = autotune.prior_order(P, 1, autotune.candidate_plans(P, 1))
    first = order[0]
    f = autotune.footprint_bytes(2, P.n, 10, first.dataflow if first.dataflow != ks.STAGED else ks.DPOB,
                                 first.chunks, 1)
    assert 2 * f <= autotune.MALL_BYTES


def test_table_lookup_exact_then_nearest_batch():
    P = FakeParams(4, 16, 32)
    key8 = autotune._cache_key(P, 8)
    table = {key8: {"plan": [ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV], "ms": 1.0, "name": "x"}}
    assert autotune.cached_plan(P, 8, table).key() == (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV, 0)
    assert autotune.cached_plan(P, 4, table) is None
    assert autotune.plan_for(P, 4, table).key() == (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV, 0)
    # entries of three-field plans (no flags) still load
    table[autotune._cache_key(P, 2)] = {"plan": [ks.DSOC, 2, 3], "ms": 1.0, "name": "y"}
    assert autotune.plan_for(P, 1, table).key() == (ks.DSOC, 2, 3, 0, 0)
    # five-field entries carry the batch tile
    table[autotune._cache_key(P, 32)] = {"plan": [ks.DPOB, 1, 4, 1, 8], "ms": 1.0, "name": "t"}
    assert autotune.cached_plan(P, 32, table).batch_tile == 8
    # flags round-trip through the table
    table[autotune._cache_key(P, 16)] = {"plan": [ks.DPOB, 1, 4, 3], "ms": 1.0, "name": "w"}
    assert autotune.cached_plan(P, 16, table).flags == ks.PLAN_MFMA_BCONV | ks.PLAN_SPLIT_STREAMS
    table[autotune._cache_key(P, 24)] = {"plan": [ks.DPOB, 1, 4, 5, 0], "ms": 1.0, "name": "h"}
    assert autotune.cached_plan(P, 24, table).flags == ks.PLAN_MFMA_BCONV | ks.PLAN_HOIST_FWD
    # another parameter set finds nothing
    assert autotune.plan_for(FakeParams(2, 15, 10), 8, table) is None
    # a stored plan the parameters do not accept is skipped
    bad = {autotune._cache_key(P, 8): {"plan": [ks.DPOB, 1, 9, ks.PLAN_MFMA_BCONV], "ms": 1.0, "name": "z"}}
    assert autotune.plan_for(P, 8, bad) is None


def test_shipped_table_entries_are_valid_plans():
    table = autotune.shipped_cache()
    assert table, "the package ships a tuning table"
    for key, e in table.items():
        assert key.count("|") == 6 and e["ms"] > 0
        f = e["plan"][3]
        p = ks.make_plan(*e["plan"][:3], bool(f & ks.PLAN_MFMA_BCONV), bool(f & ks.PLAN_SPLIT_STREAMS))
        assert p.dataflow in ks.DATAFLOW_NAMES


def test_level_handles_and_top_level_sets_get_different_keys():
    # level 16 of (4, 2^16, 32): alpha = k = 8, two digits; a top-level
    # (4, 2^16, 16) set: alpha = k = 4, four digits; different computations
    lvl = FakeParams(4, 16, 16, top_ell=32)
    top = FakeParams(4, 16, 16)
    assert (lvl.k, lvl.ndig) == (8, 2) and (top.k, top.ndig) == (4, 4)
    assert autotune._cache_key(lvl, 8) != autotune._cache_key(top, 8)
    table = {autotune._cache_key(lvl, 8): {"plan": [ks.DPOB, 1, 4, 1, 0], "ms": 1.0, "name": "lvl"}}
    assert autotune.cached_plan(lvl, 8, table) is not None
    assert autotune.cached_plan(top, 8, table) is None
    assert autotune.plan_for(top, 8, table) is None  # no fallback across shapes either
    # the shipped table has the per-level entries of (4, 2^16, 32) under k = 8
    shipped = autotune.shipped_cache()
    assert any("|dnum4|logn16|L16|k8|B8" in key for key in shipped)
    assert not any("|dnum4|logn16|L16|k4|" in key for key in shipped)
