"""Pins of the oracle's BConv, ModUp, KeyMult, ModDown and KeySwitch.

The C oracle is checked against the pure-Python oracle (defining sums) at
tiny N, against CRT-based properties at every size, and by decryption: the
KeySwitch output must decrypt under the new key to d*s within the noise bound.
Each property check is also run on a deliberately corrupted output to show
that it rejects the kind of mistake it is meant to catch.
"""
import numpy as np
import pytest

import oracle
from oracle import tiny
from synth import ciphertext_batch, uniform_residues

import pins
from conftest import CONFIGS

COLS = [0, 1, 2, 7]


def _lists(a):
    return a.tolist() if isinstance(a, np.ndarray) else a


@pytest.mark.parametrize("dnum,log_n,ell", [(2, 3, 3), (3, 3, 3), (2, 4, 4), (3, 4, 7), (1, 3, 2), (2, 5, 6)])
def test_c_oracle_equals_python_oracle(dnum, log_n, ell):
    P = oracle.Params(dnum, log_n, ell)
    T = tiny.TinyParams(dnum, log_n, ell)
    h = min(64, P.n // 2)
    s, s2, evk = oracle.keygen(P, h=h)
    ts, ts2, tevk = tiny.keygen(T, h)
    assert s.tolist() == ts and s2.tolist() == ts2
    assert evk.tolist() == tevk
    d = ciphertext_batch(P.q, P.n, 2)
    ext = oracle.modup(P, d, 2)
    acc = oracle.keymult(P, ext, evk, 2)
    out = oracle.moddown(P, acc, 2)
    assert np.array_equal(oracle.keyswitch(P, d, evk, 2), out)
    for b in range(2):
        text = tiny.modup(T, _lists(d[b]))
        assert ext[b].tolist() == text
        tacc = tiny.keymult(T, text, tevk)
        assert acc[b].tolist() == tacc
        assert out[b].tolist() == tiny.moddown(T, tacc)


@pytest.mark.parametrize("dnum,log_n,ell", [(2, 4, 6), (4, 6, 8), (3, 5, 7)])
def test_bconv_crt_property(dnum, log_n, ell):
    P = oracle.Params(dnum, log_n, ell)
    cols = list(range(P.n))
    for j in range(P.ndig):
        dig = P.digit(j)
        src = [P.moduli[i] for i in dig]
        dst = [P.moduli[t] for t in range(P.nl) if t not in dig]
        x = np.stack([uniform_residues(40 + j, [m], P.n)[0] for m in src])
        z = oracle.bconv(P, j, x[None])[0]
        assert pins.check_bconv(src, dst, x, z, cols)
        bad = z.copy()
        bad[-1, 3] = (int(bad[-1, 3]) + 1) % dst[-1]
        assert not pins.check_bconv(src, dst, x, bad, cols)
    x = uniform_residues(50, P.p, P.n)
    z = oracle.bconv(P, -1, x[None])[0]
    assert pins.check_bconv(P.p, P.q, x, z, cols)


def test_bconv_single_limb_is_exact_reduction():
    # alpha = 1 (dnum = ell): the conversion of one residue x mod q_i is x mod t
    P = oracle.Params(4, 5, 4)
    assert P.alpha == 1
    for j in range(P.ndig):
        x = uniform_residues(60 + j, [P.q[j]], P.n)
        z = oracle.bconv(P, j, x[None])[0]
        dst = [P.moduli[t] for t in range(P.nl) if t != j]
        for u, m in enumerate(dst):
            assert np.array_equal(z[u], x[0] % np.uint64(m))


def test_bconv_zero():
    P = oracle.Params(2, 5, 6)
    z = oracle.bconv(P, 1, np.zeros((1, P.alpha, P.n), dtype=np.uint64))
    assert not z.any()


@pytest.mark.parametrize("dnum,log_n,ell", [(2, 5, 6), (3, 6, 9), (4, 4, 6)])
def test_modup_keymult_moddown_properties(dnum, log_n, ell):
    P = oracle.Params(dnum, log_n, ell)
    d = ciphertext_batch(P.q, P.n, 1)
    _, _, evk = oracle.keygen(P, h=min(64, P.n // 2))
    ext = oracle.modup(P, d, 1)
    assert pins.check_modup(P, d[0], ext[0], COLS)
    acc = oracle.keymult(P, ext, evk, 1)
    assert pins.check_keymult(P, ext[0], evk, acc[0], COLS)
    out = oracle.moddown(P, acc, 1)
    assert pins.check_moddown(P, acc[0], out[0], COLS)
    # the same checks reject plausible slips
    bad = ext[0].copy()
    bad[0, P.nl - 1] = oracle.ntt(P.moduli[-1], P.psi[-1], P.log_n, np.roll(
        oracle.intt(P.moduli[-1], P.psi[-1], P.log_n, bad[0, P.nl - 1]), 1))  # transposed index
    assert not pins.check_modup(P, d[0], bad, COLS)
    bad = acc[0].copy()
    bad[[0, 1]] = bad[[1, 0]]  # components swapped
    assert not pins.check_keymult(P, ext[0], evk, bad, COLS)
    bad = out[0].copy()
    bad[0, 0] = (bad[0, 0] + np.uint64(1)) % np.uint64(P.q[0])
    assert not pins.check_moddown(P, acc[0], bad, list(range(P.n)))


def test_moddown_zero_p_part_is_exact_division():
    P = oracle.Params(2, 5, 6)
    acc = np.zeros((1, 2, P.nl, P.n), dtype=np.uint64)
    for c in range(2):
        acc[0, c, : P.ell] = uniform_residues(70 + c, P.q, P.n)
    out = oracle.moddown(P, acc, 1)
    Pbig = 1
    for p in P.p:
        Pbig *= p
    for c in range(2):
        for i, q in enumerate(P.q):
            pinv = pow(Pbig, -1, q)
            assert out[0, c, i].tolist() == [int(v) * pinv % q for v in acc[0, c, i]]


def _decrypt_case(dnum, log_n, ell, batch, h=64):
    P = oracle.Params(dnum, log_n, ell)
    h = min(h, P.n // 2)
    s, s2, evk = oracle.keygen(P, h=h)
    d = ciphertext_batch(P.q, P.n, batch)
    out = oracle.keyswitch(P, d, evk, batch)
    ok, m = pins.decrypt_ok(P, d, out, s, s2, h, batch)
    return P, s, s2, evk, d, out, ok, m


@pytest.mark.parametrize("dnum,log_n,ell", [(2, 3, 3), (3, 4, 7), (2, 10, 6), (4, 8, 8)])
def test_keyswitch_decrypts_small(dnum, log_n, ell):
    P, s, s2, evk, d, out, ok, m = _decrypt_case(dnum, log_n, ell, 2)
    assert ok, (m, oracle.ks_bound(P, min(64, P.n // 2)))
    # a wrong component order, a dropped digit or a perturbed limb fails to decrypt
    h = min(64, P.n // 2)
    assert not pins.decrypt_ok(P, d, out[:, ::-1].copy(), s, s2, h, 2)[0]
    bad = out.copy()
    bad[0, 0, 1, 5] = (bad[0, 0, 1, 5] + np.uint64(1)) % np.uint64(P.q[1])
    assert not pins.decrypt_ok(P, d, bad, s, s2, h, 2)[0]
    evk_bad = evk.copy()
    evk_bad[-1] = 0
    out_bad = oracle.keyswitch(P, d, evk_bad, 2)
    assert not pins.decrypt_ok(P, d, out_bad, s, s2, h, 2)[0]


@pytest.mark.parametrize("name", ["d2-n13-l6", "d2-n15-l10"])
def test_keyswitch_decrypts_benchmark_sizes(name):
    dnum, log_n, ell, _ = CONFIGS[name]
    P, s, s2, evk, d, out, ok, m = _decrypt_case(dnum, log_n, ell, 1)
    assert ok and m <= oracle.ks_bound(P, 64)
    assert oracle.ks_bound(P, 64) == 65 * (1 + P.k)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["d4-n16-l32", "d8-n17-l56"])
def test_keyswitch_decrypts_large(name):
    dnum, log_n, ell, _ = CONFIGS[name]
    P, s, s2, evk, d, out, ok, m = _decrypt_case(dnum, log_n, ell, 1)
    assert ok and m <= oracle.ks_bound(P, 64)


def test_keyswitch_zero_input_and_noiseless_key():
    P = oracle.Params(2, 6, 6)
    s, s2, evk = oracle.keygen(P, h=16, noiseless=True)
    d = np.zeros((1, P.ell, P.n), dtype=np.uint64)
    assert not oracle.keyswitch(P, d, evk, 1).any()
    d = ciphertext_batch(P.q, P.n, 1)
    out = oracle.keyswitch(P, d, evk, 1)
    agree, err = oracle.ks_error(P, d, out, s, s2, 1)
    # no key noise: only the ModDown terms remain, |e| < (1 + h) * k
    assert agree and int(np.abs(err).max()) < (1 + 16) * P.k


def test_keyswitch_batch_invariance():
    P = oracle.Params(3, 6, 9)
    _, _, evk = oracle.keygen(P, h=16)
    d = ciphertext_batch(P.q, P.n, 3)
    both = oracle.keyswitch(P, d, evk, 3)
    for b in range(3):
        assert np.array_equal(oracle.keyswitch(P, d[b:b + 1], evk, 1)[0], both[b])
