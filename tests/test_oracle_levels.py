"""Pins of the oracle's KeySwitch at a lower level (a ciphertext that has lost
its last limbs, switched with the top-level key): it equals the pure-Python
definition (top key restricted to the level's limbs, digits cut at the
level), reduces to the top-level KeySwitch at the top, and decrypts under the
new key within the noise bound of the level's digits."""
import numpy as np
import pytest

import oracle
from oracle import tiny
from synth import ciphertext_batch

import pins


@pytest.mark.parametrize("dnum,log_n,ell", [(2, 3, 5), (3, 4, 7), (1, 3, 3)])
def test_level_equals_python_definition(dnum, log_n, ell):
    top = oracle.Params(dnum, log_n, ell)
    T = tiny.TinyParams(dnum, log_n, ell)
    h = min(64, top.n // 2)
    _, _, evk = oracle.keygen(top, h=h)
    for level in range(1, ell + 1):
        P = top.at_level(level)
        TL = T.at_level(level)
        assert P.moduli == TL.moduli and P.psi == TL.psi and P.ndig == TL.ndig
        key = tiny.key_at_level(T, TL, evk.tolist())
        d = ciphertext_batch(P.q, P.n, 2, seed_base=70 + level)
        ext = oracle.modup(P, d, 2)
        acc = oracle.keymult(P, ext, evk, 2)
        out = oracle.moddown(P, acc, 2)
        assert np.array_equal(oracle.keyswitch(P, d, evk, 2), out)
        for b in range(2):
            text = tiny.modup(TL, d[b].tolist())
            assert ext[b].tolist() == text, (level, "modup")
            tacc = tiny.keymult(TL, text, key)
            assert acc[b].tolist() == tacc, (level, "keymult")
            assert out[b].tolist() == tiny.moddown(TL, tacc), (level, "moddown")


def test_level_at_top_is_the_top_level_keyswitch():
    P = oracle.Params(3, 6, 8)
    _, _, evk = oracle.keygen(P, h=16)
    d = ciphertext_batch(P.q, P.n, 2)
    ref = oracle.keyswitch(P, d, evk, 2)
    out = np.zeros_like(ref)
    L = oracle.lib()
    assert L.orc_keyswitch_level(P.dnum, P.log_n, P.ell, P.ell, d, evk, out, 2) == 0
    assert np.array_equal(out, ref)
    # and the level entry points reject levels outside [1, ell]
    assert L.orc_keyswitch_level(P.dnum, P.log_n, P.ell, P.ell + 1, d, evk, out, 2) != 0
    assert L.orc_keyswitch_level(P.dnum, P.log_n, P.ell, 0, d, evk, out, 2) != 0


@pytest.mark.parametrize("dnum,log_n,ell,levels", [(3, 8, 9, [1, 2, 3, 4, 5, 7, 9]), (2, 10, 6, [1, 3, 4]),
                                                   (4, 12, 16, [3, 4, 10, 13])])
def test_level_keyswitch_decrypts(dnum, log_n, ell, levels):
    top = oracle.Params(dnum, log_n, ell)
    h = min(64, top.n // 2)
    s, s2, evk = oracle.keygen(top, h=h)
    for level in levels:
        P = top.at_level(level)
        d = ciphertext_batch(P.q, P.n, 2, seed_base=300 + level)
        out = oracle.keyswitch(P, d, evk, 2)
        ok, m = pins.decrypt_ok(P, d, out, s, s2, h, 2)
        assert ok, (level, m, oracle.ks_bound(P, h))
        # the key of another level's layout, or of the wrong digit, does not decrypt
        bad = evk.copy()
        bad[0] = evk[-1]
        if P.ndig > 1:
            assert not pins.decrypt_ok(P, d, oracle.keyswitch(P, d, bad, 2), s, s2, h, 2)[0]
        # reading the P rows from the level's position instead of the top's fails
        shifted = evk.copy()
        shifted[:, :, level:level + P.k] = evk[:, :, ell:ell + P.k]
        if level < ell:
            shifted[:, :, ell:ell + P.k] = 0
            assert not pins.decrypt_ok(P, d, oracle.keyswitch(P, d, shifted, 2), s, s2, h, 2)[0]


@pytest.mark.slow
def test_level_keyswitch_decrypts_benchmark_set():
    top = oracle.Params(4, 16, 32)
    s, s2, evk = oracle.keygen(top, h=64)
    for level in (8, 21):
        P = top.at_level(level)
        d = ciphertext_batch(P.q, P.n, 1, seed_base=500 + level)
        ok, m = pins.decrypt_ok(P, d, oracle.keyswitch(P, d, evk, 1), s, s2, 64, 1)
        assert ok, (level, m)
