"""Property checks that pin the oracle to mathematics rather than to itself.

Each check reconstructs integers with the Chinese remainder theorem (Python
big integers) and tests a statement that holds for the exact KeySwitch steps
described in the paper's Background section:

* BConv: the fast conversion of x in [0, S) returns x + u*S with 0 <= u < ns;
* ModUp: the lift of digit j is an integer in [0, alpha*D_j) that is = d mod D_j;
* ModDown: the output is (A - [A]_P)/P - v with 0 <= v < k;
* KeySwitch: the output decrypts under the new key to d*s plus a small error.
"""
import math

import numpy as np

import oracle
from oracle.tiny import crt


def coeffs(P, limbs, rows):
    """INTT every row (row r over modulus P.moduli[limbs[r]]) -> python int lists."""
    out = []
    for r, t in enumerate(limbs):
        out.append([int(v) for v in oracle.intt(P.moduli[t], P.psi[t], P.log_n, rows[r])])
    return out


def check_bconv(src_mod, dst_mod, x_rows, z_rows, cols) -> bool:
    """z = BConv(x): at every sampled column, z_t = (X + u*S) mod t for one 0 <= u < len(src)."""
    S = math.prod(src_mod)
    for c in cols:
        X = crt([int(x_rows[i][c]) for i in range(len(src_mod))], src_mod)
        ok = False
        for u in range(len(src_mod)):
            v = X + u * S
            if all(int(z_rows[t][c]) == v % m for t, m in enumerate(dst_mod)):
                ok = True
                break
        if not ok:
            return False
    return True


def check_modup(P, d, ext, cols) -> bool:
    """ext = ModUp(d) for one ciphertext (d [ell][N], ext [ndig][nl][N], NTT form)."""
    dcoef = coeffs(P, list(range(P.ell)), d)
    for j in range(P.ndig):
        dig = P.digit(j)
        if not all(np.array_equal(ext[j][i], d[i]) for i in dig):
            return False
        ecoef = coeffs(P, list(range(P.nl)), ext[j])
        Dj = math.prod(P.q[i] for i in dig)
        for c in cols:
            E = crt([ecoef[t][c] for t in range(P.nl)], P.moduli)
            if not (0 <= E < len(dig) * Dj):
                return False
            if any(E % P.q[i] != dcoef[i][c] for i in dig):
                return False
    return True


def check_keymult(P, ext, evk, acc, cols) -> bool:
    """acc[c][t] = sum_j ext[j][t] * evk[j][c][t] mod t, at sampled columns."""
    for c in range(2):
        for t in range(P.nl):
            m = P.moduli[t]
            for x in cols:
                v = sum(int(ext[j][t][x]) * int(evk[j][c][t][x]) for j in range(P.ndig)) % m
                if int(acc[c][t][x]) != v:
                    return False
    return True


def check_moddown(P, acc, out, cols) -> bool:
    """out = ModDown(acc) for one ciphertext (acc [2][nl][N], out [2][ell][N])."""
    Pbig = math.prod(P.p)
    for c in range(2):
        acoef = coeffs(P, list(range(P.nl)), acc[c])
        ocoef = coeffs(P, list(range(P.ell)), out[c])
        for x in cols:
            A = crt([acoef[t][x] for t in range(P.nl)], P.moduli)
            r = A % Pbig
            base = (A - r) // Pbig
            ok = any(all(ocoef[i][x] == (base - v) % P.q[i] for i in range(P.ell)) for v in range(P.k))
            if not ok:
                return False
    return True


def decrypt_ok(P, d, out, s, s2, h, batch):
    """(ok, max|e|): every limb decrypts to the same e and |e| <= bound."""
    agree, err = oracle.ks_error(P, d, out, s, s2, batch)
    m = int(np.abs(err).max())
    return agree and m <= oracle.ks_bound(P, h), m


def _limb_decrypt(P, lhs_rows, rhs_rows):
    """(agree, max|e|) of e = INTT(lhs - rhs) over the limbs of P, as centered integers."""
    err = None
    agree = True
    for i, q in enumerate(P.q):
        diff = (lhs_rows[i].astype(object) - rhs_rows[i].astype(object)) % q
        e = oracle.intt(q, P.psi[i], P.log_n, np.array(diff, dtype=np.uint64))
        c = np.array([int(v) - q if int(v) > q // 2 else int(v) for v in e], dtype=np.int64)
        if err is None:
            err = c
        elif not np.array_equal(err, c):
            agree = False
    return agree, int(np.abs(err).max())


def _ntt_secret(P, s, i):
    q = P.q[i]
    return oracle.ntt(q, P.psi[i], P.log_n, np.array([int(v) % q for v in s], dtype=np.uint64)).astype(object)


def hmul_decrypt_ok(P, a, b, out, s, h, batch):
    """out0 + out1*s must equal (a0 + a1 s)(b0 + b1 s) up to a KeySwitch error
    within the noise bound, at every limb the same integer."""
    worst, ok = 0, True
    for bt in range(batch):
        lhs, rhs = [], []
        for i, q in enumerate(P.q):
            sh = _ntt_secret(P, s, i)
            a0, a1 = a[bt, 0, i].astype(object), a[bt, 1, i].astype(object)
            b0, b1 = b[bt, 0, i].astype(object), b[bt, 1, i].astype(object)
            lhs.append((out[bt, 0, i].astype(object) + out[bt, 1, i].astype(object) * sh) % q)
            rhs.append((a0 + a1 * sh) * (b0 + b1 * sh) % q)
        agree, m = _limb_decrypt(P, lhs, rhs)
        ok = ok and agree
        worst = max(worst, m)
    return ok and worst <= oracle.ks_bound(P, h), worst


def hrot_decrypt_ok(P, ct, g, out, s, h, batch):
    """out0 + out1*s must equal sigma_g(c0) + sigma_g(c1)*sigma_g(s) (the
    rotated ciphertext under the rotated secret), up to a KeySwitch error
    within the noise bound; sigma_g(s) is taken on the coefficients of s."""
    gs = oracle.automorph_coeffs(s, g)
    worst, ok = 0, True
    for bt in range(batch):
        lhs, rhs = [], []
        for i, q in enumerate(P.q):
            sh = _ntt_secret(P, s, i)
            gsh = _ntt_secret(P, gs, i)
            c0 = oracle.automorph(q, P.psi[i], P.log_n, ct[bt, 0, i], g).astype(object)
            c1 = oracle.automorph(q, P.psi[i], P.log_n, ct[bt, 1, i], g).astype(object)
            lhs.append((out[bt, 0, i].astype(object) + out[bt, 1, i].astype(object) * sh) % q)
            rhs.append((c0 + c1 * gsh) % q)
        agree, m = _limb_decrypt(P, lhs, rhs)
        ok = ok and agree
        worst = max(worst, m)
    return ok and worst <= oracle.ks_bound(P, h), worst
