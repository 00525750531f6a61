"""CPU oracle of the CKKS hybrid KeySwitch: test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this package. It wraps ``ks_oracle.c`` (plain C, 128-bit products reduced
with ``%``, textbook NTT loops, defining BConv sums) through ctypes, and
``tiny.py`` holds a second, pure-Python oracle for tiny N built on the O(N^2)
definition of the transform. Neither shares code with the GPU library.

The operation follows the KeySwitch description in the paper's Background
section (ModUp = iNTT -> BConv -> NTT per digit, KeyMult = multiply by the
digit's evaluation key and sum over digits, ModDown = iNTT -> BConv -> NTT then
subtract and divide by P). The choices the paper leaves open are listed in
the header of ``ks_oracle.c``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ks_oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        c_int, c_u64 = ctypes.c_int, ctypes.c_uint64
        L.orc_derive.argtypes = [c_int, c_int, c_int, _u64p, _u64p, _i64p]
        L.orc_is_prime.argtypes = [c_u64]
        L.orc_ntt.argtypes = [c_u64, c_u64, c_int, _u64p, c_int]
        L.orc_intt.argtypes = [c_u64, c_u64, c_int, _u64p, c_int]
        L.orc_bconv.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, c_int]
        L.orc_modup.argtypes = [c_int, c_int, c_int, _u64p, _u64p, c_int]
        L.orc_keymult.argtypes = [c_int, c_int, c_int, _u64p, _u64p, _u64p, c_int]
        L.orc_moddown.argtypes = [c_int, c_int, c_int, _u64p, _u64p, c_int]
        L.orc_keyswitch.argtypes = [c_int, c_int, c_int, _u64p, _u64p, _u64p, c_int]
        L.orc_keygen.argtypes = [c_int, c_int, c_int, c_int, c_u64, c_u64, c_u64, c_u64, c_int,
                                 _i8p, _i8p, _u64p]
        L.orc_ks_error.argtypes = [c_int, c_int, c_int, _u64p, _u64p, _i8p, _i8p, _i64p, c_int]
        L.orc_modup_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, c_int]
        L.orc_keymult_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, _u64p, c_int]
        L.orc_moddown_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, c_int]
        L.orc_keyswitch_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, _u64p, c_int]
        L.orc_ks_error_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, _i8p, _i8p, _i64p, c_int]
        L.orc_keygen_pair.argtypes = [c_int, c_int, c_int, _i64p, _i64p, c_u64, c_u64, c_int, _u64p]
        L.orc_automorph.argtypes = [c_u64, c_u64, c_int, _u64p, c_u64, _u64p, c_int]
        L.orc_hmul_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, _u64p, _u64p, _u64p, c_int]
        L.orc_hrot_level.argtypes = [c_int, c_int, c_int, c_int, _u64p, c_u64, _u64p, _u64p, c_int]
        L.orc_sample_ternary.argtypes = [c_u64, ctypes.c_int64, c_int, _i8p]
        L.orc_sample_gaussian.argtypes = [c_u64, ctypes.c_int64, ctypes.c_double, _i64p]
        L.orc_key_sigma.restype = ctypes.c_double
        L.orc_max_threads.restype = c_int
        L.orc_set_threads.argtypes = [c_int]
        _lib = L
    return _lib


class Params:
    """Parameters of one (dnum, N, ell) set as the oracle derives them, at
    level `level` (default: the top level ell).

    At a level l < ell the KeySwitch keeps the top level's P, k and alpha and
    works over q_0..q_{l-1} with the digits cut at l, using the top-level key
    (shape key_shape); ell, q, moduli, nl and ndig describe the level."""

    def __init__(self, dnum: int, log_n: int, ell: int, level: int = None):
        mod = np.zeros(256, dtype=np.uint64)
        psi = np.zeros(256, dtype=np.uint64)
        info = np.zeros(5, dtype=np.int64)
        if lib().orc_derive(dnum, log_n, ell, mod, psi, info) != 0:
            raise ValueError(f"invalid parameters dnum={dnum} log_n={log_n} ell={ell}")
        level = ell if level is None else level
        if not 1 <= level <= ell:
            raise ValueError(f"level {level} outside [1, {ell}]")
        self.dnum, self.log_n, self.top_ell, self.ell = dnum, log_n, ell, level
        self.n, _, self.k, self.alpha, top_ndig = (int(v) for v in info)
        top_mod = [int(v) for v in mod[: ell + self.k]]
        top_psi = [int(v) for v in psi[: ell + self.k]]
        self.moduli = top_mod[:level] + top_mod[ell:]
        self.psi = top_psi[:level] + top_psi[ell:]
        self.nl = level + self.k
        self.ndig = -(-level // self.alpha)
        self.key_shape = (top_ndig, 2, ell + self.k, self.n)
        self.q = self.moduli[: self.ell]
        self.p = self.moduli[self.ell:]

    def at_level(self, level: int) -> "Params":
        return Params(self.dnum, self.log_n, self.top_ell, level)

    def digit(self, j: int):
        lo = j * self.alpha
        return list(range(lo, min(lo + self.alpha, self.ell)))

    def __repr__(self):
        lv = f", level={self.ell}" if self.ell != self.top_ell else ""
        return f"Params(dnum={self.dnum}, N=2^{self.log_n}, ell={self.top_ell}{lv}, k={self.k})"


def _c(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(n))


def ntt(q: int, psi: int, log_n: int, a) -> np.ndarray:
    """Forward negacyclic NTT of every length-N row of a (copy returned)."""
    x = _c(a).copy()
    lib().orc_ntt(q, psi, log_n, x, x.size >> log_n)
    return x


def intt(q: int, psi: int, log_n: int, a) -> np.ndarray:
    x = _c(a).copy()
    lib().orc_intt(q, psi, log_n, x, x.size >> log_n)
    return x


def bconv(P: Params, src_set: int, src, batch: int = 1) -> np.ndarray:
    """Fast base conversion; src_set = digit j (-> PQ minus D_j) or -1 (P -> Q)."""
    src = _c(src)
    if P.ell != P.top_ell:
        raise ValueError("bconv is defined here for the top level only")
    if src_set < 0:
        nd = P.ell
    else:
        nd = P.nl - len(P.digit(src_set))
    dst = np.zeros((batch, nd, P.n), dtype=np.uint64)
    if lib().orc_bconv(P.dnum, P.log_n, P.ell, src_set, src, dst, batch) != 0:
        raise ValueError("bconv")
    return dst


def modup(P: Params, d, batch: int) -> np.ndarray:
    ext = np.zeros((batch, P.ndig, P.nl, P.n), dtype=np.uint64)
    if lib().orc_modup_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(d), ext, batch) != 0:
        raise ValueError("modup")
    return ext


def keymult(P: Params, ext, evk, batch: int) -> np.ndarray:
    """evk: the top-level key (P.key_shape)."""
    acc = np.zeros((batch, 2, P.nl, P.n), dtype=np.uint64)
    if lib().orc_keymult_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(ext), _c(evk), acc, batch) != 0:
        raise ValueError("keymult")
    return acc


def moddown(P: Params, acc, batch: int) -> np.ndarray:
    out = np.zeros((batch, 2, P.ell, P.n), dtype=np.uint64)
    if lib().orc_moddown_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(acc), out, batch) != 0:
        raise ValueError("moddown")
    return out


def keyswitch(P: Params, d, evk, batch: int) -> np.ndarray:
    """evk: the top-level key (P.key_shape); d and the output at level P.ell."""
    out = np.zeros((batch, 2, P.ell, P.n), dtype=np.uint64)
    if P.ell == P.top_ell:
        rc = lib().orc_keyswitch(P.dnum, P.log_n, P.ell, _c(d), _c(evk), out, batch)
    else:
        rc = lib().orc_keyswitch_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(d), _c(evk), out, batch)
    if rc != 0:
        raise ValueError("keyswitch")
    return out


def keygen(P: Params, h: int = 64, seeds=(1, 2, 3, 4), noiseless: bool = False):
    """(s, s2, evk): ternary secrets with h nonzeros and the key from s to s2."""
    s = np.zeros(P.n, dtype=np.int8)
    s2 = np.zeros(P.n, dtype=np.int8)
    evk = np.zeros(P.key_shape, dtype=np.uint64)  # the key is made at the top level
    rc = lib().orc_keygen(P.dnum, P.log_n, P.top_ell, h, seeds[0], seeds[1], seeds[2], seeds[3],
                          int(noiseless), s, s2, evk)
    if rc != 0:
        raise ValueError("keygen")
    return s, s2, evk


def sample_ternary(seed: int, n: int, h: int) -> np.ndarray:
    """The key generator's ternary secret: n coefficients, h of them nonzero."""
    s = np.zeros(n, dtype=np.int8)
    if lib().orc_sample_ternary(seed, n, h, s) != 0:
        raise ValueError("sample_ternary")
    return s


def sample_gaussian(seed: int, count: int, sigma: float = None) -> np.ndarray:
    """The key generator's rounded-Gaussian errors (sigma defaults to the
    keys' own, key_sigma())."""
    e = np.zeros(count, dtype=np.int64)
    if lib().orc_sample_gaussian(seed, count, key_sigma() if sigma is None else float(sigma), e) != 0:
        raise ValueError("sample_gaussian")
    return e


def key_sigma() -> float:
    """Standard deviation of the evaluation-key errors."""
    return float(lib().orc_key_sigma())


def keygen_pair(P: Params, s_from, s_to, seeds=(3, 4), noiseless: bool = False) -> np.ndarray:
    """The key from secret s_from to secret s_to (integer coefficient vectors),
    made at the top level: for instance s_from = s*s (HMUL) or sigma_g(s) (HROT)."""
    evk = np.zeros(P.key_shape, dtype=np.uint64)
    a = np.ascontiguousarray(s_from, dtype=np.int64)
    b = np.ascontiguousarray(s_to, dtype=np.int64)
    if lib().orc_keygen_pair(P.dnum, P.log_n, P.top_ell, a, b, seeds[0], seeds[1], int(noiseless), evk) != 0:
        raise ValueError("keygen_pair")
    return evk


def negacyclic_product(a, b) -> np.ndarray:
    """Integer product of two coefficient vectors in Z[x]/(x^N + 1), by the
    schoolbook sum over the nonzero coefficients of `a` (sparse secrets)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    n = len(a)
    out = np.zeros(n, dtype=np.int64)
    for i in np.nonzero(a)[0]:
        # a_i x^i * b: shift b by i, the part past x^N wraps with a sign change
        out[i:] += a[i] * b[:n - i]
        out[:i] -= a[i] * b[n - i:]
    return out


def automorph_coeffs(a, g: int) -> np.ndarray:
    """a(x) -> a(x^g) on an integer coefficient vector (g odd)."""
    a = np.asarray(a, dtype=np.int64)
    n = len(a)
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        e = (i * g) % (2 * n)
        if e < n:
            out[e] += a[i]
        else:
            out[e - n] -= a[i]
    return out


def automorph(q: int, psi: int, log_n: int, a, g: int) -> np.ndarray:
    """The automorphism x -> x^g of NTT-form limbs (rows of a), through the
    coefficient domain."""
    a = _c(a)
    out = np.zeros_like(a)
    lib().orc_automorph(q, psi, log_n, a, g, out, a.size >> log_n)
    return out


def hmul(P: Params, a, b, evk, batch: int) -> np.ndarray:
    """(a0 b0, a0 b1 + a1 b0) + KS(a1 b1); a, b, out [batch][2][level][N]."""
    out = np.zeros((batch, 2, P.ell, P.n), dtype=np.uint64)
    if lib().orc_hmul_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(a), _c(b), _c(evk), out, batch) != 0:
        raise ValueError("hmul")
    return out


def hrot(P: Params, ct, g: int, evk, batch: int) -> np.ndarray:
    """(sigma_g(c0), 0) + KS(sigma_g(c1)); ct, out [batch][2][level][N]."""
    out = np.zeros((batch, 2, P.ell, P.n), dtype=np.uint64)
    if lib().orc_hrot_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(ct), g, _c(evk), out, batch) != 0:
        raise ValueError("hrot")
    return out


def ks_error(P: Params, d, out, s, s2, batch: int):
    """(agree, err): err[b] is the decryption error of KS output b under s2
    against d*s, as centered integers; agree says every limb gives the same."""
    err = np.zeros((batch, P.n), dtype=np.int64)
    rc = lib().orc_ks_error_level(P.dnum, P.log_n, P.top_ell, P.ell, _c(d), _c(out),
                                  np.ascontiguousarray(s, np.int8), np.ascontiguousarray(s2, np.int8), err, batch)
    if rc < 0:
        raise ValueError("ks_error")
    return bool(rc), err


def ks_bound(P: Params, h: int, b_e: int = 19) -> int:
    """Largest |e| a correct KeySwitch output may show when decrypted.

    With E_j in [0, alpha*D_j) the ModUp lift of digit j, the KeySwitch output
    decrypts to d*s + W - v0 - v1*s2 where
    |W| <= sum_j N*alpha*D_j*B_e/P + 1 + h and 0 <= v_c < k, so
    |e| < sum_j N*alpha*D_j*B_e/P + (1 + h)(1 + k)."""
    from fractions import Fraction
    Pbig = 1
    for p in P.p:
        Pbig *= p
    first = Fraction(0)
    for j in range(P.ndig):
        Dj = 1
        for i in P.digit(j):
            Dj *= P.q[i]
        first += Fraction(P.n * len(P.digit(j)) * Dj * b_e, Pbig)
    import math
    return math.floor(first) + (1 + h) * (1 + P.k)
