"""Bit-exact parity of every C-ABI call of libks against the CPU oracle.

Inputs are the seeded synthetic residues of ``synth`` and keys from the
oracle's key generator; expected values come from the oracle only. Sizes
span several workgroup tiles, odd limb counts and batch sizes, every NTT
split, every dataflow, and the four benchmark parameter sets at full size.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from synth import ciphertext_batch, uniform_residues

import pins
from conftest import CONFIGS
from gpu_util import dev, empty, first_mismatch, host

pytestmark = pytest.mark.gpu

SMALL = [(3, 12, 7), (2, 10, 5), (4, 11, 8), (1, 9, 3), (3, 14, 9)]


@pytest.fixture(scope="module")
def ks():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_16692_amd as k
    return k


_params_cache = {}


def params(ks, dnum, log_n, ell):
    key = (dnum, log_n, ell)
    if key not in _params_cache:
        _params_cache[key] = (ks.KsParams(dnum, log_n, ell), oracle.Params(dnum, log_n, ell))
    return _params_cache[key]


def assert_same(gpu, ref, what):
    mm = first_mismatch(gpu, ref)
    assert mm is None, f"{what}: first mismatch {mm}"


@pytest.mark.parametrize("dnum,log_n,ell", SMALL + [v[:3] for v in CONFIGS.values()])
def test_params_match_oracle(ks, dnum, log_n, ell):
    G, P = params(ks, dnum, log_n, ell)
    assert G.moduli == P.moduli and G.psi == P.psi
    assert (G.k, G.alpha, G.ndig, G.n) == (P.k, P.alpha, P.ndig, P.n)


@pytest.mark.parametrize("dnum,log_n,ell", SMALL + [v[:3] for v in CONFIGS.values()])
def test_ntt_intt(ks, dnum, log_n, ell):
    G, P = params(ks, dnum, log_n, ell)
    batch = 3 if log_n < 16 else 1
    x = np.stack([uniform_residues(11 + b, P.moduli, P.n) for b in range(batch)])
    ref_f = np.empty_like(x)
    ref_i = np.empty_like(x)
    for b in range(batch):
        for t in range(P.nl):
            ref_f[b, t] = oracle.ntt(P.moduli[t], P.psi[t], log_n, x[b, t])
            ref_i[b, t] = oracle.intt(P.moduli[t], P.psi[t], log_n, x[b, t])
    y = dev(x)
    G.ntt(y, 0, P.nl, batch)
    assert_same(host(y), ref_f, "ntt")
    y = dev(x)
    G.intt(y, 0, P.nl, batch)
    assert_same(host(y), ref_i, "intt")
    # a sub-range of the basis: the P limbs only
    y = dev(np.ascontiguousarray(x[:, P.ell:]))
    G.ntt(y, P.ell, P.k, batch)
    assert_same(host(y), ref_f[:, P.ell:], "ntt on P limbs")


@pytest.mark.parametrize("dnum,log_n,ell", SMALL + [v[:3] for v in CONFIGS.values()])
def test_bconv(ks, dnum, log_n, ell):
    G, P = params(ks, dnum, log_n, ell)
    batch = 2
    for j in list(range(P.ndig)) + [-1]:
        src_mod = P.p if j < 0 else [P.moduli[i] for i in P.digit(j)]
        x = np.stack([uniform_residues(30 + b + 3 * j, src_mod, P.n) for b in range(batch)])
        ref = oracle.bconv(P, j, x, batch)
        out = empty(ref.shape)
        G.bconv(dev(x), j, out, batch)
        assert_same(host(out), ref, f"bconv set {j}")


@pytest.mark.parametrize("dnum,log_n,ell", SMALL + [(2, 13, 6), (2, 15, 10), (4, 16, 32)])
def test_modup_keymult_moddown(ks, dnum, log_n, ell):
    G, P = params(ks, dnum, log_n, ell)
    batch = 3 if log_n < 16 else 1
    d = ciphertext_batch(P.q, P.n, batch)
    _, _, evk = oracle.keygen(P, h=min(64, P.n // 2))
    ext_ref = oracle.modup(P, d, batch)
    acc_ref = oracle.keymult(P, ext_ref, evk, batch)
    out_ref = oracle.moddown(P, acc_ref, batch)
    ws = G.workspace(batch, ks.make_plan(ks.STAGED))
    ext = empty(ext_ref.shape)
    G.modup(dev(d), ext, batch, ws)
    assert_same(host(ext), ext_ref, "modup")
    acc = empty(acc_ref.shape)
    G.keymult(dev(ext_ref), dev(evk), acc, batch)
    assert_same(host(acc), acc_ref, "keymult")
    acc_in = dev(acc_ref)
    out = empty(out_ref.shape)
    G.moddown(acc_in, out, batch, ws)
    assert_same(host(out), out_ref, "moddown")
    assert_same(host(acc_in), acc_ref, "moddown leaves acc unchanged")


def _plans(ks, P, log_n):
    plans = []
    for log_r in range(0, 6):
        log_m = log_n - log_r
        if log_m < 3 or log_m > 14:
            continue
        for df, chunks in [(ks.DSOB, 1), (ks.DPOB, 1), (ks.DSOC, 2), (ks.DPOC, 3), (ks.STAGED, 1)]:
            chunks = min(chunks, P.ell)
            plans.append(ks.make_plan(df, chunks, log_r))
            plans.append(ks.make_plan(df, chunks, log_r, mfma=True))  # the int8-MFMA BConv
            # the batch over two streams (3 items: 1 + 2)
            plans.append(ks.make_plan(df, chunks, log_r, mfma=True, split=True))
            # passes of 2 + 1 items reusing one workspace, and of 1 item
            plans.append(ks.make_plan(df, chunks, log_r, tile=2))
            if df == ks.DPOB:  # the raised digits' forward pass as a launch of its own
                plans.append(ks.make_plan(df, chunks, log_r, hoist=True))
                plans.append(ks.make_plan(df, chunks, log_r, mfma=True, split=True, hoist=True))
            if log_r == 3:
                plans.append(ks.make_plan(df, chunks, log_r, mfma=True, split=True, tile=2))
                plans.append(ks.make_plan(df, chunks, log_r, tile=1))
    return plans


@pytest.mark.parametrize("dnum,log_n,ell", SMALL)
def test_keyswitch_every_plan(ks, dnum, log_n, ell):
    G, P = params(ks, dnum, log_n, ell)
    batch = 3
    d = ciphertext_batch(P.q, P.n, batch)
    _, _, evk = oracle.keygen(P, h=min(64, P.n // 2))
    ref = oracle.keyswitch(P, d, evk, batch)
    dd, ee = dev(d), dev(evk)
    for plan in _plans(ks, P, log_n):
        out = empty(ref.shape)
        ws = G.workspace(batch, plan)
        G.keyswitch(dd, ee, out, batch, ws, plan)
        assert_same(host(out), ref, f"keyswitch {plan}")


_full_cache = {}


def full_case(ks, name):
    if name not in _full_cache:
        dnum, log_n, ell, batch = CONFIGS[name]
        G, P = params(ks, dnum, log_n, ell)
        s, s2, evk = oracle.keygen(P, h=64)
        d = ciphertext_batch(P.q, P.n, batch)
        ref = oracle.keyswitch(P, d, evk, batch)
        _full_cache[name] = (G, P, s, s2, evk, d, ref, batch)
    return _full_cache[name]


@pytest.mark.parametrize("name", ["d2-n13-l6", "d2-n15-l10", "d4-n16-l32", "d8-n17-l56"])
def test_keyswitch_benchmark_sizes(ks, name):
    G, P, s, s2, evk, d, ref, batch = full_case(ks, name)
    dd, ee = dev(d), dev(evk)
    plans = [None, ks.make_plan(ks.DSOB), ks.make_plan(ks.DPOC, 4), ks.make_plan(ks.DSOC, 2),
             ks.make_plan(ks.DPOB, 1, 4, mfma=True), ks.make_plan(ks.DSOC, 3, 3, mfma=True),
             ks.make_plan(ks.STAGED, 1, 4, mfma=True), ks.make_plan(ks.DPOB, 1, 4, mfma=True, split=True),
             ks.make_plan(ks.DPOB, 1, 5, mfma=True), ks.make_plan(ks.DPOB, 1, 4, mfma=True, tile=3),
             ks.make_plan(ks.DPOB, 1, 4, mfma=True, hoist=True)]
    for plan in plans:
        out = empty(ref.shape)
        ws = G.workspace(batch, plan)
        G.keyswitch(dd, ee, out, batch, ws, plan)
        got = host(out)
        assert_same(got, ref, f"{name} keyswitch {plan}")
        del ws, out
    ok, m = pins.decrypt_ok(P, d, got, s, s2, 64, batch)
    assert ok, f"decryption error {m} above bound {oracle.ks_bound(P, 64)}"


def test_keyswitch_deep_set_one_ciphertext(ks):
    # (8, 2^17, 56) with one ciphertext at the top level, under the tuned
    # plan of the shipped table, DSOB, the library default and two others;
    # the oracle computes the items of a batch one by one, so the reference
    # of item 0 is that of the batch case
    from paper_2603_16692_amd import autotune
    G, P, s, s2, evk, d, ref, _ = full_case(ks, "d8-n17-l56")
    d1 = np.ascontiguousarray(d[:1])
    ref1 = oracle.keyswitch(P, d1, evk, 1)
    assert np.array_equal(ref1, ref[:1])
    tuned = autotune.plan_for(G, 1, autotune.shipped_cache())
    assert tuned is not None
    dd, ee = dev(d1), dev(evk)
    for plan in (tuned, ks.make_plan(ks.DSOB), None, ks.make_plan(ks.DSOB, 1, 5, mfma=True),
                 ks.make_plan(ks.DPOC, 4, 4, mfma=True), ks.make_plan(ks.STAGED, 1, 5, mfma=True),
                 ks.make_plan(ks.DPOB, 1, 5, mfma=True, hoist=True)):
        out = empty(ref1.shape)
        G.keyswitch(dd, ee, out, 1, G.workspace(1, plan), plan)
        got = host(out)
        assert_same(got, ref1, f"d8-n17-l56 batch 1 {plan}")
    ok, m = pins.decrypt_ok(P, d1, got, s, s2, 64, 1)
    assert ok, m


def test_batch_item_equals_single(ks):
    G, P = params(ks, 3, 12, 7)
    d = ciphertext_batch(P.q, P.n, 5)
    _, _, evk = oracle.keygen(P, h=64)
    dd, ee = dev(d), dev(evk)
    out = empty((5, 2, P.ell, P.n))
    G.keyswitch(dd, ee, out, 5, G.workspace(5))
    allb = host(out)
    for b in range(5):
        one = empty((1, 2, P.ell, P.n))
        G.keyswitch(dev(d[b:b + 1]), ee, one, 1, G.workspace(1))
        assert_same(host(one)[0], allb[b], f"item {b}")


def test_two_streams_concurrently(ks):
    G, P = params(ks, 2, 15, 10)
    d = ciphertext_batch(P.q, P.n, 4)
    _, _, evk = oracle.keygen(P, h=64)
    ref = oracle.keyswitch(P, d, evk, 4)
    ee = dev(evk)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs, keep = [], []
    for i, st in enumerate(streams):
        with torch.cuda.stream(st):
            dd = dev(d[2 * i:2 * i + 2])
            ws = G.workspace(2)
            out = empty((2, 2, P.ell, P.n))
            for _ in range(3):
                G.keyswitch(dd, ee, out, 2, ws, stream=st)
            outs.append(out)
            keep += [dd, ws]
    torch.cuda.synchronize()
    for i in range(2):
        assert_same(host(outs[i]), ref[2 * i:2 * i + 2], f"stream {i}")


def test_zero_input_gives_zero(ks):
    G, P = params(ks, 2, 13, 6)
    _, _, evk = oracle.keygen(P, h=64)
    d = np.zeros((2, P.ell, P.n), dtype=np.uint64)
    out = empty((2, 2, P.ell, P.n))
    G.keyswitch(dev(d), dev(evk), out, 2, G.workspace(2))
    assert not host(out).any()


def test_argument_errors(ks):
    G, P = params(ks, 2, 13, 6)
    ws = G.workspace(1)
    d = empty((1, P.ell, P.n))
    evk = empty((P.ndig, 2, P.nl, P.n))
    out = empty((1, 2, P.ell, P.n))
    with pytest.raises(ValueError):  # the binding refuses a missing buffer itself
        G.keyswitch(d, evk, None, 1, ws)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ks.raw_call("ks_keyswitch", G._h, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(evk.data_ptr()), None, 1,
                     None, ctypes.c_void_p(ws.data_ptr()), stream)
    assert rc == ks.KS_ENULL
    bad = empty(P.ell * P.n + 1)[1:]
    with pytest.raises(ks.KsError) as e:
        G.keyswitch(bad, evk, out, 1, ws)
    assert e.value.code == ks.KS_EALIGN
    with pytest.raises(ks.KsError) as e:
        G.keyswitch(d, evk, out, 1, ws, ks.make_plan(ks.DSOC, 0))
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:
        G.keyswitch(d, evk, out, 1, ws, ks.make_plan(ks.DPOB, 1, 9))
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:  # 32 rows of 12 sources exceed the MFMA BConv's LDS
        ks.KsParams(1, 12, 12).workspace_bytes(1, ks.make_plan(ks.DPOB, 1, 5, mfma=True))
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:  # ... and at most 16 sources per BConv
        ks.KsParams(1, 10, 20).workspace_bytes(1, ks.make_plan(ks.DPOB, 1, 2, mfma=True))
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:
        G.keyswitch(d, evk, out, 1, ws, ks.Plan(ks.DPOB, 1, 2, 8))  # an unknown flag bit
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:  # the hoisted forward pass with a dataflow other than DPOB
        G.keyswitch(d, evk, out, 1, ws, ks.Plan(ks.DSOC, 2, 2, ks.PLAN_HOIST_FWD))
    assert e.value.code == ks.KS_EUNSUP
    with pytest.raises(ks.KsError) as e:
        G.ntt(d, P.nl - 1, 2, 1)
    assert e.value.code == ks.KS_EINVAL
    with pytest.raises(ks.KsError) as e:
        G.bconv(d, P.ndig, out, 1)
    assert e.value.code == ks.KS_EINVAL
    with pytest.raises(ks.KsError) as e:
        ks.KsParams(3, 13, 2)
    assert e.value.code == ks.KS_EINVAL
    with pytest.raises(ks.KsError) as e:
        ks.KsParams(1, 18, 2)
    assert e.value.code == ks.KS_EINVAL
    # batch 0 is a no-op
    G.keyswitch(d, evk, out, 0, ws)


def _expected_launches(P, df, c):
    """Kernel launches of the plan executor: the KeyMult stage starts one
    kernel for the Q limbs of its target range and one for the P limbs;
    digit-parallel plans leave the Q limbs to ModDown's last pass."""
    def chunks(n):
        return [(n * i // c, n * (i + 1) // c) for i in range(c) if n * i // c < n * (i + 1) // c]

    def km(a, b, q):
        return int(q and a < min(b, P.ell)) + int(max(a, P.ell) < b)
    n = 1
    for a, b in chunks(P.nl):
        if df in ("DPOB", "DPOC"):
            n += 1 + km(a, b, False)
        else:
            n += P.ndig * (1 + km(a, b, True))
    return n + 2 * len(chunks(P.ell))


def test_launch_counts_follow_table_iii(ks):
    # Table III: launches DSOB O(d), DPOB O(1), DSOC O(dc), DPOC O(c)
    G, P = params(ks, 4, 16, 32)
    assert G.launch_count(1, ks.make_plan(ks.DPOB)) == 5 == _expected_launches(P, "DPOB", 1)
    assert G.launch_count(1, ks.make_plan(ks.DPOB, hoist=True)) == 6  # the raised digits' forward pass on its own
    with pytest.raises(ks.KsError) as e:  # the hoisted forward pass exists for DPOB only
        G.workspace_bytes(1, ks.make_plan(ks.DSOB, hoist=True))
    assert e.value.code == ks.KS_EUNSUP
    assert G.launch_count(1, ks.make_plan(ks.DSOB)) == _expected_launches(P, "DSOB", 1) == 1 + 3 * P.ndig + 2
    for c in (2, 3, 5):
        assert G.launch_count(1, ks.make_plan(ks.DPOC, c)) == _expected_launches(P, "DPOC", c)
        assert G.launch_count(1, ks.make_plan(ks.DSOC, c)) == _expected_launches(P, "DSOC", c)
    # scaling: DP plans do not grow with dnum, DS plans do; OC plans grow with chunks
    G8, P8 = params(ks, 8, 13, 32)
    assert G8.launch_count(1, ks.make_plan(ks.DPOB)) == G.launch_count(1, ks.make_plan(ks.DPOB))
    assert G8.launch_count(1, ks.make_plan(ks.DSOB)) > G.launch_count(1, ks.make_plan(ks.DSOB))
    assert G.launch_count(1, ks.make_plan(ks.DPOC, 6)) > G.launch_count(1, ks.make_plan(ks.DPOC, 3))
    # a split batch runs each plan twice (once per half), a batch of one is not split
    sp = ks.make_plan(ks.DPOB, split=True)
    assert G.launch_count(4, sp) == 2 * G.launch_count(4, ks.make_plan(ks.DPOB))
    assert G.launch_count(1, sp) == G.launch_count(1, ks.make_plan(ks.DPOB))
    assert G.workspace_bytes(5, sp) == G.workspace_bytes(2) + G.workspace_bytes(3)
    # a tiled batch runs one pass per tile in the workspace of one tile
    tp = ks.make_plan(ks.DPOB, tile=3)
    assert G.launch_count(8, tp) == 3 * G.launch_count(1, ks.make_plan(ks.DPOB))
    assert G.workspace_bytes(8, tp) == G.workspace_bytes(3) < G.workspace_bytes(8)
    assert G.launch_count(8, ks.make_plan(ks.DPOB, split=True, tile=3)) == 6 * 5
    with pytest.raises(ks.KsError) as e:
        G.workspace_bytes(8, ks.make_plan(ks.DPOB, tile=-1))
    assert e.value.code == ks.KS_EUNSUP


def test_default_plan_valid_for_large_digits(ks):
    # alpha = 25: the default NTT split is reduced until the column kernels can stage the digit
    for dnum, log_n, ell in ((2, 16, 50), (2, 17, 50), (1, 12, 30)):
        G = ks.KsParams(dnum, log_n, ell)
        p = G.default_plan(1)
        assert G.workspace_bytes(1, p) > 0 and p.log_r >= 0
    G, P = params(ks, 1, 12, 30)
    d = ciphertext_batch(P.q, P.n, 1)
    _, _, evk = oracle.keygen(P, h=64)
    out = empty((1, 2, P.ell, P.n))
    G.keyswitch(dev(d), dev(evk), out, 1, G.workspace(1))
    assert_same(host(out), oracle.keyswitch(P, d, evk, 1), "alpha = 30")


@pytest.mark.parametrize("dnum,log_n,ell,batch", [
    (2, 10, 85, 1),   # ell + k = 128 limbs, the most the library takes; 43-prime digits
    (6, 11, 6, 2),    # alpha = 1: every digit one prime, BConv an exact reduction
    (1, 10, 12, 1),   # one digit holding every Q limb
    (2, 3, 4, 3),     # N = 8, the smallest ring
    (4, 12, 13, 2),   # ragged digits 4, 4, 4, 1
])
def test_extreme_shapes(ks, dnum, log_n, ell, batch):
    G, P = params(ks, dnum, log_n, ell)
    d = ciphertext_batch(P.q, P.n, batch)
    _, _, evk = oracle.keygen(P, h=min(64, P.n // 2))
    ref = oracle.keyswitch(P, d, evk, batch)
    for plan in (None, ks.make_plan(ks.STAGED), ks.make_plan(ks.DSOB), ks.make_plan(ks.DPOB, hoist=True)):
        out = empty(ref.shape)
        G.keyswitch(dev(d), dev(evk), out, batch, G.workspace(batch, plan), plan)
        assert_same(host(out), ref, f"{(dnum, log_n, ell)} {plan}")


def test_limits_are_rejected_on_the_host(ks):
    # checked before anything is enqueued: no kernel sees these sizes
    for args in ((2, 10, 86), (1, 18, 4), (1, 2, 4), (5, 12, 4), (0, 12, 4)):
        with pytest.raises(ks.KsError) as e:
            ks.KsParams(*args)
        assert e.value.code == ks.KS_EINVAL, args
    G, P = params(ks, 2, 13, 6)
    d = empty((1, P.ell, P.n))
    out = empty((1, 2, P.ell, P.n))
    evk = empty((P.ndig, 2, P.nl, P.n))
    with pytest.raises(ValueError):  # the binding sees that the buffers hold one item
        G.keyswitch(d, evk, out, 40000, G.workspace(1))
    with pytest.raises(ks.KsError) as e:
        G.keyswitch(d, evk, out, -1, G.workspace(1))
    assert e.value.code == ks.KS_EINVAL
    # straight through the C ABI, whose limits are checked before anything is
    # enqueued: batch * max(2, ndig) above 65535 grid rows, products that wrap
    # in 32 bits (2^30 * 2, 2^29 * 8), more than 2^31 coefficients per call
    ws = G.workspace(1)
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (d, evk, out)]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for batch in (40000, 1 << 29, 1 << 30, (1 << 31) - 1, -5):
        rc = ks.raw_call("ks_keyswitch", G._h, *ptrs, batch, None, ctypes.c_void_p(ws.data_ptr()), stream)
        assert rc == ks.KS_EINVAL, batch
        rc = ks.raw_call("ks_hmul", G._h, ptrs[0], ptrs[0], ptrs[1], ptrs[2], batch, None,
                         ctypes.c_void_p(ws.data_ptr()), stream)
        assert rc == ks.KS_EINVAL, batch
        rc = ks.raw_call("ks_modup", G._h, ptrs[0], ptrs[2], batch, ctypes.c_void_p(ws.data_ptr()), stream)
        assert rc == ks.KS_EINVAL, batch
        rc = ks.raw_call("ks_moddown", G._h, ptrs[2], ptrs[2], batch, ctypes.c_void_p(ws.data_ptr()), stream)
        assert rc == ks.KS_EINVAL, batch
        rc = ks.raw_call("ks_ntt", G._h, ptrs[0], 0, P.nl, batch, stream)
        assert rc == ks.KS_EINVAL, batch
    big, _ = params(ks, 8, 17, 56)
    # (ell + k) * N = 63 * 2^17 coefficients per item: 261 items exceed 2^31 in one call
    dummy = ctypes.c_void_p(ws.data_ptr())
    assert ks.raw_call("ks_keyswitch", big._h, dummy, dummy, dummy, 261, None, dummy, stream) == ks.KS_EINVAL
    torch.cuda.synchronize()
