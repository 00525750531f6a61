"""Pins of the oracle's parameter derivation (primes, psi).

Primality is proven independently of the oracle's Miller-Rabin by a Lucas
certificate (a full factorisation of q-1 and a witness of order q-1), and the
"largest primes" rule by a Fermat or small-factor witness of compositeness
for every skipped candidate.
"""
import pytest
import sympy

import oracle
from oracle import tiny

from conftest import CONFIGS


def lucas_certificate(q: int) -> bool:
    """q is prime iff some a has order q-1 mod q (Lucas' theorem)."""
    fac = sympy.factorint(q - 1)
    for a in range(2, 200):
        if pow(a, q - 1, q) != 1:
            return False
        if all(pow(a, (q - 1) // f, q) != 1 for f in fac):
            return True
    return False


def composite_witness(c: int) -> bool:
    """True when c is shown composite by a small factor or a Fermat witness."""
    for p in (3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47):
        if c % p == 0:
            return True
    return any(pow(a, c - 1, c) != 1 for a in (2, 3, 5, 7, 11))


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_primes_rule(name):
    dnum, log_n, ell, _ = CONFIGS[name]
    P = oracle.Params(dnum, log_n, ell)
    two_n = 2 * P.n
    assert P.k == P.alpha == -(-ell // dnum)
    assert len(set(P.moduli)) == P.nl
    for q in P.q:
        assert 2 ** 49 <= q < 2 ** 50 and q % two_n == 1
    for p in P.p:
        assert 2 ** 59 <= p < 2 ** 60 and p % two_n == 1
    for group, bits in ((P.q, 50), (P.p, 60)):
        assert group == sorted(group, reverse=True)
        # every candidate = 1 mod 2N between 2^bits and the last prime taken is
        # either taken (and proven prime) or proven composite
        c = ((2 ** bits - 1) // two_n) * two_n + 1
        taken = set(group)
        while c >= group[-1]:
            if c in taken:
                assert lucas_certificate(c), c
            else:
                assert composite_witness(c), c
            c -= two_n


@pytest.mark.parametrize("log_n,ell,dnum", [(3, 3, 3), (4, 5, 2), (6, 4, 4), (10, 6, 2)])
def test_derivation_matches_independent_rule(log_n, ell, dnum):
    P = oracle.Params(dnum, log_n, ell)
    T = tiny.TinyParams(dnum, log_n, ell)
    assert P.moduli == T.moduli
    assert P.psi == T.psi
    assert (P.k, P.alpha, P.ndig) == (T.k, T.alpha, T.ndig)


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_psi_is_smallest_primitive_root(name):
    dnum, log_n, ell, _ = CONFIGS[name]
    P = oracle.Params(dnum, log_n, ell)
    n = P.n
    # every limb: psi is a primitive 2N-th root of unity
    for m, psi in zip(P.moduli, P.psi):
        assert pow(psi, n, m) == m - 1
    # minimality against the full root set of x^N + 1, on one Q and one P prime
    for t in (0, P.nl - 1):
        m = P.moduli[t]
        g = None
        for x in range(2, 100):
            c = pow(x, (m - 1) // (2 * n), m)
            if pow(c, n, m) == m - 1:
                g = c
                break
        g2, cur, best = g * g % m, g, g
        seen = 0
        for _ in range(n):
            best = min(best, cur)
            cur = cur * g2 % m
            seen += 1
        assert seen == n and P.psi[t] == best


def test_uneven_digits():
    # ell = 10, dnum = 6 -> alpha = 2, five digits, k = 2
    P = oracle.Params(6, 4, 10)
    assert (P.alpha, P.k, P.ndig) == (2, 2, 5)
    assert [P.digit(j) for j in range(P.ndig)] == [[0, 1], [2, 3], [4, 5], [6, 7], [8, 9]]
    # ell = 7, dnum = 3 -> alpha = 3, last digit short
    P = oracle.Params(3, 4, 7)
    assert (P.alpha, P.ndig) == (3, 3) and P.digit(2) == [6]


def test_invalid_parameters():
    with pytest.raises(ValueError):
        oracle.Params(5, 4, 3)  # dnum > ell
    with pytest.raises(ValueError):
        oracle.Params(1, 0, 3)
