"""Pins of the oracle's key samplers against their definitions.

The evaluation keys of every parity and decryption test come from two
samplers: a ternary secret with exactly h nonzero coefficients in {-1, +1}
(h = 64, or N/2 at tiny N) and rounded-Gaussian key errors of standard
deviation 3.2, cut at |e| <= 19. The paper states neither sampler; these
tests check the oracle's against the definitions themselves (exact counts,
ranges, the moments and the probability mass function of the rounded normal,
uniformity of positions and signs), not against a second implementation, and
tie the key generator to the samplers by recovering the secrets and errors
from a key. Each check is also shown to reject a planted slip: one nonzero
too few, a coefficient out of range, a one-signed secret, sigma = 1.6.
"""
import math

import numpy as np
import pytest

import oracle

H = 64
SIGMA = 3.2
CUT = 19


def check_ternary(s, h) -> bool:
    """Exactly h nonzeros, every coefficient in {-1, 0, +1}."""
    s = np.asarray(s, dtype=np.int64)
    return bool(np.all(np.abs(s) <= 1)) and int(np.count_nonzero(s)) == h


def both_signs(s) -> bool:
    s = np.asarray(s, dtype=np.int64)
    return bool(np.any(s == 1) and np.any(s == -1))


def rounded_normal_pmf(sigma, cut):
    """P(round(sigma*z) = v | |round(sigma*z)| <= cut) for v = -cut..cut."""
    def phi(x):
        return 0.5 * (1.0 + math.erf(x / (sigma * math.sqrt(2.0))))
    p = np.array([phi(v + 0.5) - phi(v - 0.5) for v in range(-cut, cut + 1)])
    return p / p.sum()


def gaussian_ok(e, sigma=SIGMA, cut=CUT) -> bool:
    """The sample is the rounded normal of the given sigma, cut at `cut`:
    range, mean, standard deviation and a chi-square fit of the mass function
    (bins with an expected count below 50 are merged into the tails)."""
    e = np.asarray(e, dtype=np.int64)
    n = len(e)
    if int(np.abs(e).max()) > cut:
        return False
    pmf = rounded_normal_pmf(sigma, cut)
    mean_pmf = 0.0
    std_pmf = math.sqrt(float(np.sum(pmf * np.arange(-cut, cut + 1) ** 2)))
    if abs(float(e.mean()) - mean_pmf) > 6 * std_pmf / math.sqrt(n):
        return False
    if abs(float(e.std()) - std_pmf) > 0.05:
        return False
    counts = np.bincount(e + cut, minlength=2 * cut + 1).astype(float)
    exp = pmf * n
    keep = exp >= 50
    lo = int(np.argmax(keep))
    hi = len(keep) - int(np.argmax(keep[::-1]))
    obs = np.concatenate([[counts[:lo].sum()], counts[lo:hi], [counts[hi:].sum()]])
    ex = np.concatenate([[exp[:lo].sum()], exp[lo:hi], [exp[hi:].sum()]])
    m = ex > 0
    chi2 = float(np.sum((obs[m] - ex[m]) ** 2 / ex[m]))
    dof = int(m.sum()) - 1
    # mean dof, standard deviation sqrt(2 dof): accept up to six deviations
    return chi2 < dof + 6 * math.sqrt(2 * dof)


@pytest.mark.parametrize("log_n", [3, 4, 6, 10, 13, 15, 16, 17])
def test_ternary_has_exactly_h_signed_ones(log_n):
    n = 1 << log_n
    h = min(H, n // 2)
    for seed in [1, 2] + list(range(100, 140)):
        s = oracle.sample_ternary(seed, n, h)
        assert check_ternary(s, h), (seed, n)
        if h >= 16:
            assert both_signs(s), (seed, n)


def test_ternary_check_rejects_planted_slips():
    s = oracle.sample_ternary(1, 1 << 13, H)
    assert check_ternary(s, H)
    short = s.copy()
    short[np.flatnonzero(short)[0]] = 0  # h - 1 nonzeros
    assert not check_ternary(short, H)
    wide = s.copy()
    wide[np.flatnonzero(wide)[0]] = 2  # a coefficient outside {-1, 0, 1}
    assert not check_ternary(wide, H)
    assert not both_signs(np.abs(s))  # a sampler that never draws -1


def test_ternary_signs_and_positions_are_uniform():
    n, reps = 1024, 2000
    total_plus, hist = 0, np.zeros(n)
    for seed in range(10_000, 10_000 + reps):
        s = oracle.sample_ternary(seed, n, H)
        nz = np.flatnonzero(s)
        total_plus += int(np.sum(s[nz] == 1))
        hist[nz] += 1
    draws = reps * H
    # signs: Binomial(draws, 1/2), six standard deviations
    assert abs(total_plus - draws / 2) < 6 * math.sqrt(draws) / 2
    # positions: each of n slots equally likely (chi-square, n - 1 dof)
    exp = draws / n
    chi2 = float(np.sum((hist - exp) ** 2 / exp))
    assert chi2 < (n - 1) + 6 * math.sqrt(2 * (n - 1))
    # planted: positions confined to the first half fail the same statistic
    bad = np.zeros(n)
    bad[: n // 2] = draws / (n // 2)
    assert float(np.sum((bad - exp) ** 2 / exp)) > (n - 1) + 6 * math.sqrt(2 * (n - 1))


def test_keygen_secrets_are_the_sampler_outputs():
    for dnum, log_n, ell in [(2, 13, 6), (2, 5, 4), (3, 3, 3)]:
        P = oracle.Params(dnum, log_n, ell)
        h = min(H, P.n // 2)
        s, s2, _ = oracle.keygen(P, h=h)
        assert np.array_equal(s, oracle.sample_ternary(1, P.n, h))
        assert np.array_equal(s2, oracle.sample_ternary(2, P.n, h))
        assert check_ternary(s, h) and check_ternary(s2, h)


def test_gaussian_is_the_rounded_normal_of_sigma_3_2():
    assert oracle.key_sigma() == SIGMA
    e = oracle.sample_gaussian(4, 200_000)
    assert int(np.abs(e).max()) <= CUT
    assert abs(float(e.std()) - SIGMA) < 0.05
    assert gaussian_ok(e)
    # another seed
    assert gaussian_ok(oracle.sample_gaussian(99, 150_000))


def test_gaussian_check_rejects_planted_slips():
    # the sampler run with half the standard deviation
    half = oracle.sample_gaussian(4, 200_000, sigma=1.6)
    assert int(np.abs(half).max()) <= CUT
    assert not gaussian_ok(half)
    # the right sigma but a one-sided (biased) sample
    e = oracle.sample_gaussian(4, 200_000)
    assert not gaussian_ok(np.abs(e))
    # values past the cut
    wide = e.copy()
    wide[0] = CUT + 1
    assert not gaussian_ok(wide)
    # every value off by one (a rounding slip that moves the mean)
    assert not gaussian_ok(e - 1)


def _centered(v, q):
    v = int(v)
    return v - q if v > q // 2 else v


def _key_errors(P, s, s2, evk):
    """e_j recovered from the key at every limb: INTT(b + a*s2 - [t in D_j] P s)."""
    Pbig = math.prod(P.p)
    errs = []
    for j in range(P.ndig):
        dig = P.digit(j)
        per_limb = []
        for t, m in enumerate(P.moduli):
            sh = oracle.ntt(m, P.psi[t], P.log_n, np.array([int(v) % m for v in s], dtype=np.uint64))
            s2h = oracle.ntt(m, P.psi[t], P.log_n, np.array([int(v) % m for v in s2], dtype=np.uint64))
            b = evk[j, 0, t].astype(object)
            a = evk[j, 1, t].astype(object)
            eh = (b + a * s2h.astype(object)) % m
            if t in dig:
                eh = (eh - (Pbig % m) * sh.astype(object)) % m
            e = oracle.intt(m, P.psi[t], P.log_n, np.array(eh, dtype=np.uint64))
            per_limb.append([_centered(v, m) for v in e])
        errs.append(per_limb)
    return errs


def test_key_carries_the_sampled_errors_on_every_limb():
    P = oracle.Params(2, 8, 4)
    s, s2, evk = oracle.keygen(P, h=H)
    want = oracle.sample_gaussian(4, P.ndig * P.n)
    errs = _key_errors(P, s, s2, evk)
    for j in range(P.ndig):
        for t in range(P.nl):
            assert errs[j][t] == want[j * P.n:(j + 1) * P.n].tolist(), (j, t)
    # planted: a noiseless key carries no error, which the same recovery shows
    _, _, clean = oracle.keygen(P, h=H, noiseless=True)
    errs0 = _key_errors(P, s, s2, clean)
    assert all(v == 0 for j in range(P.ndig) for t in range(P.nl) for v in errs0[j][t])
    assert any(v != 0 for v in want)
