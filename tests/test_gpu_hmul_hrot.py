"""Bit-exact parity of ks_hmul and ks_hrot (the ciphertext product with
relinearisation, and the slot rotation) against the oracle, at the top level
and at lower levels, under several KeySwitch plans, and by decryption at a
benchmark size."""
import numpy as np
import pytest
import torch

import oracle
from synth import ciphertext_batch

import pins
from gpu_util import dev, empty, first_mismatch, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_16692_amd as k
    return k


def _ct(P, batch, seed):
    return ciphertext_batch(P.q, P.n, 2 * batch, seed_base=seed).reshape(batch, 2, P.ell, P.n)


def assert_same(gpu, ref, what):
    mm = first_mismatch(gpu, ref)
    assert mm is None, f"{what}: first mismatch {mm}"


@pytest.mark.parametrize("dnum,log_n,ell,levels", [(3, 12, 7, [7, 3]), (2, 10, 5, [5, 1]), (4, 13, 16, [16, 9])])
def test_hmul_and_hrot_match_oracle(ks, dnum, log_n, ell, levels):
    top = ks.KsParams(dnum, log_n, ell)
    Pt = oracle.Params(dnum, log_n, ell)
    s, _, _ = oracle.keygen(Pt, h=64)
    mk = dev(oracle.keygen_pair(Pt, oracle.negacyclic_product(s, s), s))
    batch = 3
    for level in levels:
        G = top.at_level(level) if level != ell else top
        P = Pt.at_level(level)
        a, b = _ct(P, batch, 10 + level), _ct(P, batch, 20 + level)
        ref = oracle.hmul(P, a, b, host(mk).reshape(P.key_shape), batch)
        # fused plans fold the tensor product into the KeySwitch's first and
        # last passes (digit-parallel and digit-serial last passes, split
        # batches); STAGED runs it as separate kernels
        for plan in (None, ks.make_plan(ks.DPOB, 1, 2, mfma=True), ks.make_plan(ks.DSOC, min(2, level), 3),
                     ks.make_plan(ks.DSOB, 1, 0), ks.make_plan(ks.DPOC, min(2, level), 1, split=True),
                     ks.make_plan(ks.STAGED), ks.make_plan(ks.DPOB, 1, 2, tile=2), ks.make_plan(ks.STAGED, tile=2),
                     ks.make_plan(ks.DPOB, 1, 2, mfma=True, hoist=True)):
            out = empty(ref.shape)
            G.hmul(dev(a), dev(b), mk, out, batch, G.eval_workspace(batch, plan), plan)
            assert_same(host(out), ref, f"hmul level {level} {plan}")
        hrot_plans = (ks.make_plan(ks.DPOB, 1, 2, mfma=True), ks.make_plan(ks.DSOC, min(2, level), 3),
                      ks.make_plan(ks.DPOC, min(2, level), 1, split=True), ks.make_plan(ks.STAGED),
                      ks.make_plan(ks.DPOB, 1, 2, tile=2), ks.make_plan(ks.DPOB, 1, 2, split=True, hoist=True))
        for gi, g in enumerate((5, 25, 2 * P.n - 1)):
            rk_h = oracle.keygen_pair(Pt, oracle.automorph_coeffs(s, g), s)
            ref = oracle.hrot(P, a, g, rk_h, batch)
            # sigma_g is folded into the KeySwitch's first and last passes
            # under the fused plans, separate kernels under STAGED
            for plan in (hrot_plans if gi == 0 else hrot_plans[:1]):
                out = empty(ref.shape)
                G.hrot(dev(a), g, dev(rk_h), out, batch, G.eval_workspace(batch, plan), plan)
                assert_same(host(out), ref, f"hrot g={g} level {level} {plan}")


def test_hrot_rejects_bad_galois_elements(ks):
    G = ks.KsParams(2, 10, 5)
    ct = empty((1, 2, 5, 1 << 10))
    out = empty((1, 2, 5, 1 << 10))
    evk = empty(G.shapes(1)["evk"])
    ws = G.eval_workspace(1)
    for g in (0, 4, 2048, 2049, -3):
        with pytest.raises(ks.KsError) as e:
            G.hrot(ct, g, evk, out, 1, ws)
        assert e.value.code == ks.KS_EINVAL


def test_hmul_hrot_decrypt_at_benchmark_size(ks):
    dnum, log_n, ell, batch = 2, 15, 10, 2
    G = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    s, _, _ = oracle.keygen(P, h=64)
    mk = oracle.keygen_pair(P, oracle.negacyclic_product(s, s), s)
    a, b = _ct(P, batch, 31), _ct(P, batch, 32)
    plan = ks.make_plan(ks.DPOB, 1, 3, mfma=True)
    out = empty((batch, 2, ell, P.n))
    G.hmul(dev(a), dev(b), dev(mk), out, batch, G.eval_workspace(batch, plan), plan)
    got = host(out)
    assert_same(got, oracle.hmul(P, a, b, mk, batch), "hmul")
    ok, m = pins.hmul_decrypt_ok(P, a, b, got, s, 64, batch)
    assert ok, m
    g = 5 ** 3 % (2 * P.n)
    rk = oracle.keygen_pair(P, oracle.automorph_coeffs(s, g), s)
    G.hrot(dev(a), g, dev(rk), out, batch, G.eval_workspace(batch, plan), plan)
    got = host(out)
    assert_same(got, oracle.hrot(P, a, g, rk, batch), "hrot")
    ok, m = pins.hrot_decrypt_ok(P, a, g, got, s, 64, batch)
    assert ok, m


def test_hmul_hrot_headline_set_batch8(ks):
    # (4, 2^16, 32), batch 8, under the shipped plan of this set (DPOB, log_r 4,
    # int8-MFMA BConv) with the tensor product / automorphism fused, under
    # STAGED with them as kernels of their own, and under the hoisted DPOB
    from paper_2603_16692_amd import autotune
    dnum, log_n, ell, batch = 4, 16, 32, 8
    G = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    shipped = autotune.plan_for(G, batch, autotune.shipped_cache())
    assert shipped is not None and shipped.key()[:4] == (ks.DPOB, 1, 4, ks.PLAN_MFMA_BCONV)
    s, _, _ = oracle.keygen(P, h=64)
    mk = oracle.keygen_pair(P, oracle.negacyclic_product(s, s), s)
    a, b = _ct(P, batch, 41), _ct(P, batch, 42)
    da, db, dk = dev(a), dev(b), dev(mk)
    ref = oracle.hmul(P, a, b, mk, batch)
    out = empty(ref.shape)
    plans = (shipped, ks.make_plan(ks.STAGED, 1, 4, mfma=True), ks.make_plan(ks.DPOB, 1, 4, mfma=True, hoist=True))
    for plan in plans:
        out.zero_()
        G.hmul(da, db, dk, out, batch, G.eval_workspace(batch, plan), plan)
        got = host(out)
        assert_same(got, ref, f"hmul (4, 2^16, 32) b8 {plan}")
    ok, m = pins.hmul_decrypt_ok(P, a[:1], b[:1], got[:1], s, 64, 1)
    assert ok, m
    g = 5 ** 7 % (2 * P.n)
    rk = oracle.keygen_pair(P, oracle.automorph_coeffs(s, g), s)
    ref = oracle.hrot(P, a, g, rk, batch)
    drk = dev(rk)
    for plan in plans:
        out.zero_()
        G.hrot(da, g, drk, out, batch, G.eval_workspace(batch, plan), plan)
        got = host(out)
        assert_same(got, ref, f"hrot (4, 2^16, 32) b8 {plan}")
    ok, m = pins.hrot_decrypt_ok(P, a[:1], g, got[:1], s, 64, 1)
    assert ok, m
