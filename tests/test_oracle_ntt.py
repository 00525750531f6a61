"""Pins of the oracle's negacyclic NTT / INTT.

* the fast loop equals the O(N^2) defining sum (pure Python) for N <= 256;
* the convolution theorem against schoolbook multiplication in Z_q[x]/(x^N+1);
* INTT(NTT(a)) = a at every benchmark size;
* closed forms at full size: NTT(1) = 1 everywhere, NTT(x^j)[t] = psi^(j*(2*brv(t)+1)).
"""
import numpy as np
import pytest

import oracle
from oracle import tiny
from synth import uniform_residues

from conftest import CONFIGS


@pytest.mark.parametrize("log_n", [1, 2, 3, 5, 8])
def test_fast_ntt_equals_definition(log_n):
    P = oracle.Params(2, log_n, 3)
    for t in (0, P.ell):  # one Q prime, one P prime
        q, psi = P.moduli[t], P.psi[t]
        a = uniform_residues(17 + log_n, [q], P.n)[0]
        A = oracle.ntt(q, psi, log_n, a)
        assert [int(v) for v in A] == tiny.ntt_def([int(v) for v in a], q, psi, log_n)
        back = oracle.intt(q, psi, log_n, A)
        assert [int(v) for v in back] == tiny.intt_def([int(v) for v in A], q, psi, log_n)
        assert np.array_equal(back, a)


@pytest.mark.parametrize("log_n", [2, 4, 6])
def test_convolution_theorem(log_n):
    P = oracle.Params(2, log_n, 3)
    for t in range(P.nl):
        q, psi = P.moduli[t], P.psi[t]
        a = uniform_residues(5, [q], P.n)[0]
        b = uniform_residues(6, [q], P.n)[0]
        prod = oracle.intt(q, psi, log_n, [(int(x) * int(y)) % q for x, y in zip(oracle.ntt(q, psi, log_n, a),
                                                                             oracle.ntt(q, psi, log_n, b))])
        ref = tiny.negacyclic_mul([int(v) for v in a], [int(v) for v in b], q)
        assert [int(v) for v in prod] == ref


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_roundtrip_and_closed_forms(name):
    dnum, log_n, ell, _ = CONFIGS[name]
    P = oracle.Params(dnum, log_n, ell)
    n = P.n
    rng = np.random.default_rng(0)
    for t in (0, ell - 1, ell, P.nl - 1):
        q, psi = P.moduli[t], P.psi[t]
        a = uniform_residues(99, [q], n)[0]
        assert np.array_equal(oracle.intt(q, psi, log_n, oracle.ntt(q, psi, log_n, a)), a)
        one = np.zeros(n, dtype=np.uint64)
        one[0] = 1
        assert np.all(oracle.ntt(q, psi, log_n, one) == 1)
        for j in (1, 3, n - 1):
            mono = np.zeros(n, dtype=np.uint64)
            mono[j] = 1
            A = oracle.ntt(q, psi, log_n, mono)
            for s in rng.integers(0, n, size=64):
                s = int(s)
                assert int(A[s]) == pow(psi, j * (2 * tiny.brv(s, log_n) + 1), q)
        # x^N = -1: shifting by one place multiplies slot t by psi^(2 brv(t) + 1)
        shifted = np.roll(a, 1)
        shifted[0] = (q - int(a[-1])) % q
        A, B = oracle.ntt(q, psi, log_n, a), oracle.ntt(q, psi, log_n, shifted)
        for s in rng.integers(0, n, size=64):
            s = int(s)
            assert int(B[s]) == int(A[s]) * pow(psi, 2 * tiny.brv(s, log_n) + 1, q) % q
