"""Bit-exact parity of the level-aware KeySwitch (ks_params_at_level): a
ciphertext that has lost its last limbs, switched with the top-level key,
against the oracle at the same level, for every step, several plans, levels
that cut a digit, fill it exactly or keep a single limb, and the benchmark
parameter sets."""
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


def assert_same(gpu, ref, what):
    mm = first_mismatch(gpu, ref)
    assert mm is None, f"{what}: first mismatch {mm}"


def test_level_handle_parameters(ks):
    top = ks.KsParams(3, 12, 7)
    P = oracle.Params(3, 12, 7)
    for level in range(1, 8):
        G = top.at_level(level)
        L = P.at_level(level)
        assert G.ell == level and G.key_ell == 7 and G.k == P.k and G.alpha == P.alpha
        assert G.ndig == L.ndig and G.moduli == L.moduli and G.psi == L.psi
        assert G.shapes(2)["evk"] == P.key_shape
    for bad in (0, 8, -1):
        with pytest.raises(ks.KsError) as e:
            top.at_level(bad)
        assert e.value.code == ks.KS_EINVAL


@pytest.mark.parametrize("dnum,log_n,ell,levels", [(3, 12, 7, [1, 2, 3, 4, 5, 6]), (2, 10, 5, [1, 3, 4]),
                                                   (4, 11, 8, [2, 5]), (3, 14, 9, [4, 7])])
def test_level_keyswitch_every_plan(ks, dnum, log_n, ell, levels):
    top = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    _, _, evk = oracle.keygen(P, h=64)
    ee = dev(evk)
    batch = 3
    for level in levels:
        G = top.at_level(level)
        L = P.at_level(level)
        d = ciphertext_batch(L.q, L.n, batch, seed_base=40 + level)
        ref = oracle.keyswitch(L, d, evk, batch)
        dd = dev(d)
        c = min(2, level)  # chunks of the output limbs, at most one per limb
        plans = [None, ks.make_plan(ks.DSOB), ks.make_plan(ks.DPOC, c), ks.make_plan(ks.STAGED),
                 ks.make_plan(ks.DPOB, 1, 2, mfma=True), ks.make_plan(ks.DSOC, c, 3, mfma=True, split=True),
                 ks.make_plan(ks.DPOB, 1, 2, hoist=True)]
        for plan in plans:
            out = empty(ref.shape)
            G.keyswitch(dd, ee, out, batch, G.workspace(batch, plan), plan)
            assert_same(host(out), ref, f"level {level} {plan}")


def test_level_steps(ks):
    top = ks.KsParams(3, 12, 7)
    P = oracle.Params(3, 12, 7)
    _, _, evk = oracle.keygen(P, h=64)
    batch = 2
    for level in (2, 5):
        G = top.at_level(level)
        L = P.at_level(level)
        d = ciphertext_batch(L.q, L.n, batch, seed_base=90 + level)
        ext_ref = oracle.modup(L, d, batch)
        acc_ref = oracle.keymult(L, ext_ref, evk, batch)
        out_ref = oracle.moddown(L, acc_ref, batch)
        ws = G.workspace(batch, ks.make_plan(ks.STAGED))
        ext = empty(ext_ref.shape)
        G.modup(dev(d), ext, batch, ws)
        assert_same(host(ext), ext_ref, f"modup level {level}")
        acc = empty(acc_ref.shape)
        G.keymult(dev(ext_ref), dev(evk), acc, batch)
        assert_same(host(acc), acc_ref, f"keymult level {level}")
        out = empty(out_ref.shape)
        G.moddown(dev(acc_ref), out, batch, ws)
        assert_same(host(out), out_ref, f"moddown level {level}")


@pytest.mark.parametrize("dnum,log_n,ell,batch,levels", [(2, 15, 10, 8, [3, 7]), (4, 16, 32, 2, [8, 21]),
                                                         (8, 17, 56, 1, [30])])
def test_level_benchmark_sets(ks, dnum, log_n, ell, batch, levels):
    top = ks.KsParams(dnum, log_n, ell)
    P = oracle.Params(dnum, log_n, ell)
    s, s2, evk = oracle.keygen(P, h=64)
    ee = dev(evk)
    for level in levels:
        G = top.at_level(level)
        L = P.at_level(level)
        d = ciphertext_batch(L.q, L.n, batch, seed_base=700 + level)
        ref = oracle.keyswitch(L, d, evk, batch)
        for plan in (ks.make_plan(ks.DPOB, 1, 4, mfma=True), ks.make_plan(ks.DSOB, 1, 3)):
            out = empty(ref.shape)
            G.keyswitch(dev(d), ee, out, batch, G.workspace(batch, plan), plan)
            got = host(out)
            assert_same(got, ref, f"level {level} {plan}")
        ok, m = pins.decrypt_ok(L, d, got, s, s2, 64, batch)
        assert ok, (level, m)
