"""Second oracle for tiny N, in pure Python integers (test infrastructure).

It shares nothing with ``ks_oracle.c`` except the published definitions:
the transform here is the O(N^2) defining sum, not a butterfly loop, the
primes are tested with sympy, psi is the minimum of the explicitly listed
root set of x^N + 1, and every step of the KeySwitch (Background section,
"KeySwitch" subsection) is written from its definition. It is used to check
the C oracle bit for bit at N <= 256 and to check its pins (CRT, schoolbook
negacyclic convolution).
"""
import math

import sympy

from synth import splitmix64


def brv(x: int, bits: int) -> int:
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def primes_desc(bits: int, two_n: int, count: int):
    """The `count` largest primes below 2^bits that are = 1 (mod 2N), descending."""
    out = []
    c = ((2 ** bits - 1) // two_n) * two_n + 1
    while len(out) < count:
        if sympy.isprime(c):
            out.append(c)
        c -= two_n
    return out


def root_set(q: int, n: int):
    """All roots of x^N + 1 modulo the prime q (the primitive 2N-th roots)."""
    for x in range(2, q):
        g = pow(x, (q - 1) // (2 * n), q)
        if pow(g, n, q) == q - 1:
            break
    roots = {pow(g, e, q) for e in range(1, 2 * n, 2)}
    assert len(roots) == n and all(pow(r, n, q) == q - 1 for r in roots)
    return roots


def smallest_psi(q: int, n: int) -> int:
    return min(root_set(q, n))


class TinyParams:
    def __init__(self, dnum: int, log_n: int, ell: int):
        self.dnum, self.log_n, self.ell = dnum, log_n, ell
        self.n = 1 << log_n
        self.alpha = -(-ell // dnum)
        self.k = self.alpha
        self.ndig = -(-ell // self.alpha)
        self.q = primes_desc(50, 2 * self.n, ell)
        self.p = primes_desc(60, 2 * self.n, self.k)
        self.moduli = self.q + self.p
        self.nl = len(self.moduli)
        self.psi = [smallest_psi(m, self.n) for m in self.moduli]

    def digit(self, j):
        lo = j * self.alpha
        return list(range(lo, min(lo + self.alpha, self.ell)))

    def at_level(self, level: int) -> "TinyParams":
        """The set at `level` Q limbs: the first `level` primes of Q, the same
        P, k and alpha, the digits cut at `level`."""
        L = TinyParams.__new__(TinyParams)
        L.__dict__.update(self.__dict__)
        L.top_ell = self.ell
        L.ell = level
        L.q = self.q[:level]
        L.moduli = L.q + L.p
        L.psi = self.psi[:level] + self.psi[self.ell:]
        L.nl = len(L.moduli)
        L.ndig = -(-level // self.alpha)
        return L


def key_at_level(top: TinyParams, L: TinyParams, evk):
    """The top-level key restricted to the limbs of level L: digits j < L.ndig,
    rows of q_0..q_{level-1} and of P."""
    rows = list(range(L.ell)) + [top.ell + m for m in range(top.k)]
    return [[[list(evk[j][c][r]) for r in rows] for c in range(2)] for j in range(L.ndig)]


def ntt_def(a, q: int, psi: int, log_n: int):
    """NTT(a)[t] = sum_i a_i * psi^(i*(2*brv(t)+1)) mod q."""
    n = 1 << log_n
    out = []
    for t in range(n):
        r = pow(psi, 2 * brv(t, log_n) + 1, q)
        s, rp = 0, 1
        for i in range(n):
            s += a[i] * rp
            rp = rp * r % q
        out.append(s % q)
    return out


def intt_def(A, q: int, psi: int, log_n: int):
    """a_i = N^-1 * sum_t A[t] * psi^(-i*(2*brv(t)+1)) mod q."""
    n = 1 << log_n
    ninv = pow(n, -1, q)
    pinv = pow(psi, -1, q)
    out = []
    for i in range(n):
        s = 0
        for t in range(n):
            s += A[t] * pow(pinv, i * (2 * brv(t, log_n) + 1), q)
        out.append(s * ninv % q)
    return out


def negacyclic_mul(a, b, q: int):
    """Schoolbook product in Z_q[x]/(x^N + 1)."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return [v % q for v in c]


def crt(residues, moduli) -> int:
    """The integer in [0, prod(moduli)) with the given residues."""
    M = math.prod(moduli)
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += r * Mi * pow(Mi, -1, m)
    return x % M


def bconv_def(x_rows, src_mod, dst_mod):
    """Fast base conversion of coefficient rows x_rows[i][c] (mod src_mod[i])."""
    S = math.prod(src_mod)
    n = len(x_rows[0])
    y = [[x_rows[i][c] * pow(S // src_mod[i], -1, src_mod[i]) % src_mod[i] for c in range(n)]
         for i in range(len(src_mod))]
    out = []
    for t in dst_mod:
        out.append([sum(y[i][c] * (S // src_mod[i]) for i in range(len(src_mod))) % t for c in range(n)])
    return out


def modup(P: TinyParams, d):
    """d[ell][N] NTT form -> ext[ndig][nl][N] NTT form."""
    ext = []
    for j in range(P.ndig):
        dig = P.digit(j)
        x = [intt_def(d[i], P.moduli[i], P.psi[i], P.log_n) for i in dig]
        others = [t for t in range(P.nl) if t not in dig]
        z = bconv_def(x, [P.moduli[i] for i in dig], [P.moduli[t] for t in others])
        row = [None] * P.nl
        for u, t in enumerate(others):
            row[t] = ntt_def(z[u], P.moduli[t], P.psi[t], P.log_n)
        for i in dig:
            row[i] = list(d[i])
        ext.append(row)
    return ext


def keymult(P: TinyParams, ext, evk):
    acc = [[[0] * P.n for _ in range(P.nl)] for _ in range(2)]
    for c in range(2):
        for t in range(P.nl):
            m = P.moduli[t]
            for x in range(P.n):
                acc[c][t][x] = sum(ext[j][t][x] * evk[j][c][t][x] for j in range(P.ndig)) % m
    return acc


def moddown(P: TinyParams, acc):
    out = []
    Pbig = math.prod(P.p)
    for c in range(2):
        xs = [intt_def(acc[c][P.ell + m], P.p[m], P.psi[P.ell + m], P.log_n) for m in range(P.k)]
        z = bconv_def(xs, P.p, P.q)
        row = []
        for i in range(P.ell):
            q = P.q[i]
            zh = ntt_def(z[i], q, P.psi[i], P.log_n)
            pinv = pow(Pbig, -1, q)
            row.append([(acc[c][i][x] - zh[x]) * pinv % q for x in range(P.n)])
        out.append(row)
    return out


def keyswitch(P: TinyParams, d, evk):
    return moddown(P, keymult(P, modup(P, d), evk))


def _draw(seed: int, idx: int) -> int:
    return int(splitmix64(seed, idx, 1)[0])


def ternary(seed: int, n: int, h: int):
    perm = list(range(n))
    s = [0] * n
    idx = 0
    for i in range(h):
        r = _draw(seed, idx); idx += 1
        j = i + r % (n - i)
        perm[i], perm[j] = perm[j], perm[i]
        r2 = _draw(seed, idx); idx += 1
        s[perm[i]] = 1 if (r2 & 1) else -1
    return s


def gaussian(seed: int, count: int):
    out, idx = [], 0
    for _ in range(count):
        while True:
            u1 = ((_draw(seed, idx) >> 11) + 1.0) * 2.0 ** -53; idx += 1
            u2 = (_draw(seed, idx) >> 11) * 2.0 ** -53; idx += 1
            z = math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)
            v = round(3.2 * z)  # round half to even, as nearbyint in the default mode
            if abs(v) <= 19:
                out.append(v)
                break
    return out


def keygen(P: TinyParams, h: int, seeds=(1, 2, 3, 4), noiseless: bool = False):
    s = ternary(seeds[0], P.n, h)
    s2 = ternary(seeds[1], P.n, h)
    e = [0] * (P.ndig * P.n) if noiseless else gaussian(seeds[3], P.ndig * P.n)
    Pbig = math.prod(P.p)
    evk = []
    for j in range(P.ndig):
        dig = P.digit(j)
        bj, aj = [], []
        for t in range(P.nl):
            m = P.moduli[t]
            sh = ntt_def([v % m for v in s], m, P.psi[t], P.log_n)
            s2h = ntt_def([v % m for v in s2], m, P.psi[t], P.log_n)
            eh = ntt_def([v % m for v in e[j * P.n:(j + 1) * P.n]], m, P.psi[t], P.log_n)
            a = [int(v) % m for v in splitmix64(seeds[2], (j * P.nl + t) * P.n, P.n)]
            own = Pbig % m if t in dig else 0
            bj.append([(-a[x] * s2h[x] + eh[x] + own * sh[x]) % m for x in range(P.n)])
            aj.append(a)
        evk.append([bj, aj])
    return s, s2, evk


def keygen_pair(P: TinyParams, s_from, s_to, seeds=(3, 4), noiseless: bool = False):
    """The key from s_from to s_to (integer coefficient lists), as keygen."""
    e = [0] * (P.ndig * P.n) if noiseless else gaussian(seeds[1], P.ndig * P.n)
    Pbig = math.prod(P.p)
    evk = []
    for j in range(P.ndig):
        dig = P.digit(j)
        bj, aj = [], []
        for t in range(P.nl):
            m = P.moduli[t]
            sh = ntt_def([v % m for v in s_from], m, P.psi[t], P.log_n)
            s2h = ntt_def([v % m for v in s_to], m, P.psi[t], P.log_n)
            eh = ntt_def([v % m for v in e[j * P.n:(j + 1) * P.n]], m, P.psi[t], P.log_n)
            a = [int(v) % m for v in splitmix64(seeds[0], (j * P.nl + t) * P.n, P.n)]
            own = Pbig % m if t in dig else 0
            bj.append([(-a[x] * s2h[x] + eh[x] + own * sh[x]) % m for x in range(P.n)])
            aj.append(a)
        evk.append([bj, aj])
    return evk


def automorph_poly(a, g: int):
    """a(x) -> a(x^g) in Z[x]/(x^N + 1) on a coefficient list."""
    n = len(a)
    out = [0] * n
    for i, v in enumerate(a):
        e = i * g % (2 * n)
        if e < n:
            out[e] += v
        else:
            out[e - n] -= v
    return out


def hmul(P: TinyParams, a, b, evk):
    """a = (a0, a1), b = (b0, b1) NTT-form lists over Q:
    (a0 b0, a0 b1 + a1 b0) + KS(a1 b1)."""
    n = P.n
    d0 = [[a[0][i][x] * b[0][i][x] % P.q[i] for x in range(n)] for i in range(P.ell)]
    d1 = [[(a[0][i][x] * b[1][i][x] + a[1][i][x] * b[0][i][x]) % P.q[i] for x in range(n)] for i in range(P.ell)]
    d2 = [[a[1][i][x] * b[1][i][x] % P.q[i] for x in range(n)] for i in range(P.ell)]
    ks = keyswitch(P, d2, evk)
    return [[[(d[i][x] + ks[c][i][x]) % P.q[i] for x in range(n)] for i in range(P.ell)]
            for c, d in enumerate((d0, d1))]


def hrot(P: TinyParams, ct, g: int, evk):
    """(sigma_g(c0), 0) + KS(sigma_g(c1)), sigma_g computed on coefficients."""
    def sigma(rows):
        out = []
        for i in range(P.ell):
            q = P.q[i]
            coeffs = intt_def(rows[i], q, P.psi[i], P.log_n)
            out.append(ntt_def([v % q for v in automorph_poly(coeffs, g)], q, P.psi[i], P.log_n))
        return out
    c0, c1 = sigma(ct[0]), sigma(ct[1])
    ks = keyswitch(P, c1, evk)
    return [[[(c0[i][x] + ks[0][i][x]) % P.q[i] for x in range(P.n)] for i in range(P.ell)], ks[1]]

