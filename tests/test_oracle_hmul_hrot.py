"""Pins of the oracle's HMUL and HROT (the next rows after the KeySwitch):
the automorphism against its closed forms and the ring structure, both
operations against the pure-Python definitions at tiny N, and both by
decryption (the output must decrypt to the product, or to the rotated
ciphertext under the rotated secret, within the KeySwitch noise bound)."""
import numpy as np
import pytest

import oracle
from oracle import tiny
from synth import ciphertext_batch, uniform_residues

import pins


def _ct(P, batch, seed):
    """batch ciphertexts [batch][2][ell][N], uniform in NTT form."""
    c = ciphertext_batch(P.q, P.n, 2 * batch, seed_base=seed)
    return c.reshape(batch, 2, P.ell, P.n)


def _brv(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2)


@pytest.mark.parametrize("log_n", [3, 5, 8])
def test_automorph_closed_forms_and_ring_structure(log_n):
    P = oracle.Params(2, log_n, 2)
    q, psi, n = P.q[0], P.psi[0], P.n
    a = uniform_residues(11, [q], n)[0]
    b = uniform_residues(12, [q], n)[0]
    aut = lambda x, g: oracle.automorph(q, psi, log_n, x, g)
    assert np.array_equal(aut(a, 1), a)
    for g, h in [(5, 3), (2 * n - 1, 5), (25, 2 * n - 5)]:
        assert np.array_equal(aut(aut(a, h), g), aut(a, g * h % (2 * n)))
        prod = (a.astype(object) * b.astype(object) % q).astype(np.uint64)
        lhs = aut(prod, g)
        rhs = (aut(a, g).astype(object) * aut(b, g).astype(object) % q).astype(np.uint64)
        assert np.array_equal(lhs, rhs), "not a ring homomorphism"
        # in NTT form the automorphism permutes the evaluation points:
        # slot t holds a(psi^(2brv(t)+1)), so sigma_g(a) at t is a at the slot of g*(2brv(t)+1)
        perm = [_brv((g * (2 * _brv(t, log_n) + 1) % (2 * n) - 1) // 2, log_n) for t in range(n)]
        assert np.array_equal(aut(a, g), a[perm])
    # x -> x^(2N-1) = x^-1: coefficient i goes to -(N - i), the constant stays
    c = oracle.intt(q, psi, log_n, a)
    conj = np.zeros(n, dtype=object)
    conj[0] = int(c[0])
    for i in range(1, n):
        conj[n - i] = (q - int(c[i])) % q
    assert np.array_equal(oracle.intt(q, psi, log_n, aut(a, 2 * n - 1)), conj.astype(np.uint64))


@pytest.mark.parametrize("dnum,log_n,ell,level", [(2, 3, 3, 3), (3, 4, 7, 7), (3, 4, 7, 4), (1, 3, 2, 2)])
def test_hmul_and_hrot_equal_python_definitions(dnum, log_n, ell, level):
    top = oracle.Params(dnum, log_n, ell)
    T = tiny.TinyParams(dnum, log_n, ell)
    P, TL = top.at_level(level), T.at_level(level)
    h = min(64, top.n // 2)
    s, _, _ = oracle.keygen(top, h=h)
    s2 = oracle.negacyclic_product(s, s)
    evk = oracle.keygen_pair(top, s2, s)
    tevk = tiny.keygen_pair(T, s2.tolist(), s.tolist())
    assert evk.tolist() == tevk
    a, b = _ct(P, 2, 50), _ct(P, 2, 60)
    out = oracle.hmul(P, a, b, evk, 2)
    key = tiny.key_at_level(T, TL, tevk)
    for bt in range(2):
        assert out[bt].tolist() == tiny.hmul(TL, a[bt].tolist(), b[bt].tolist(), key)
    g = 5
    gs = oracle.automorph_coeffs(s, g)
    assert gs.tolist() == tiny.automorph_poly(s.tolist(), g)
    rk = oracle.keygen_pair(top, gs, s)
    rout = oracle.hrot(P, a, g, rk, 2)
    rkey = tiny.key_at_level(T, TL, rk.tolist())
    for bt in range(2):
        assert rout[bt].tolist() == tiny.hrot(TL, a[bt].tolist(), g, rkey)


def test_negacyclic_product_matches_schoolbook():
    n = 16
    rng = np.random.default_rng(3)
    a = rng.integers(-1, 2, n)
    b = rng.integers(-5, 6, n)
    q = (1 << 61) - 1
    ref = tiny.negacyclic_mul([int(v) % q for v in a], [int(v) % q for v in b], q)
    got = oracle.negacyclic_product(a, b)
    assert [int(v) % q for v in got] == ref


@pytest.mark.parametrize("dnum,log_n,ell,levels", [(3, 10, 7, [7, 4]), (2, 13, 6, [6]), (2, 15, 10, [10, 3])])
def test_hmul_decrypts(dnum, log_n, ell, levels):
    top = oracle.Params(dnum, log_n, ell)
    h = 64
    s, _, _ = oracle.keygen(top, h=h)
    evk = oracle.keygen_pair(top, oracle.negacyclic_product(s, s), s)
    for level in levels:
        P = top.at_level(level)
        a, b = _ct(P, 1, 80 + level), _ct(P, 1, 90 + level)
        out = oracle.hmul(P, a, b, evk, 1)
        ok, m = pins.hmul_decrypt_ok(P, a, b, out, s, h, 1)
        assert ok, (level, m, oracle.ks_bound(P, h))
        # swapped inputs give the same product; a perturbed output does not decrypt
        assert np.array_equal(oracle.hmul(P, b, a, evk, 1), out)
        bad = out.copy()
        bad[0, 1, 0, 3] = (bad[0, 1, 0, 3] + np.uint64(1)) % np.uint64(P.q[0])
        assert not pins.hmul_decrypt_ok(P, a, b, bad, s, h, 1)[0]


@pytest.mark.parametrize("dnum,log_n,ell,gs", [(3, 10, 7, [5, 25, 2047]), (2, 13, 6, [5, 16383])])
def test_hrot_decrypts(dnum, log_n, ell, gs):
    top = oracle.Params(dnum, log_n, ell)
    h = 64
    s, _, _ = oracle.keygen(top, h=h)
    P = top
    ct = _ct(P, 1, 120)
    for g in gs:
        rk = oracle.keygen_pair(top, oracle.automorph_coeffs(s, g), s)
        out = oracle.hrot(P, ct, g, rk, 1)
        ok, m = pins.hrot_decrypt_ok(P, ct, g, out, s, h, 1)
        assert ok, (g, m)
        # the key of another rotation does not decrypt
        wrong = oracle.keygen_pair(top, oracle.automorph_coeffs(s, 3), s)
        assert not pins.hrot_decrypt_ok(P, ct, g, oracle.hrot(P, ct, g, wrong, 1), s, h, 1)[0]
