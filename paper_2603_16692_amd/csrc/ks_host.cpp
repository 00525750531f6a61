// Host-side derivation of the parameters of one (dnum, N, ell) set and of
// every constant table the kernels read.
//
// Parameter rules (the paper leaves them open): Q holds the ell largest
// primes below 2^50 and P the k = alpha largest primes below 2^60, all
// = 1 (mod 2N), in descending order; psi is the smallest primitive 2N-th root
// of unity modulo each prime; alpha = ceil(ell / dnum).
#include "ks_host.hpp"

#include <algorithm>
#include <cstring>

namespace ks {

using u128 = unsigned __int128;

uint64_t host_mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t host_powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m, x = a % m;
  for (; e; e >>= 1) {
    if (e & 1) r = host_mulmod(r, x, m);
    x = host_mulmod(x, x, m);
  }
  return r;
}

namespace {

uint64_t inv_prime(uint64_t a, uint64_t p) { return host_powmod(a, p - 2, p); }

// Strong probable-prime test to every base in {2..37}; exact below 3.3e24.
bool strong_prime(uint64_t n) {
  if (n < 2) return false;
  const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  int s = __builtin_ctzll(n - 1);
  uint64_t d = (n - 1) >> s;
  for (uint64_t a : small) {
    uint64_t x = host_powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s && witness; ++r) {
      x = host_mulmod(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

bool largest_primes(int bits, uint64_t step, int count, std::vector<uint64_t>& out) {
  const uint64_t limit = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
  uint64_t c = limit - (limit % step) + 1;  // largest value = 1 (mod step) not above limit + 1
  if (c > limit) c -= step;
  for (int got = 0; got < count; c -= step) {
    if (c <= step) return false;
    if (strong_prime(c)) {
      out.push_back(c);
      ++got;
    }
  }
  return true;
}

uint64_t smallest_root(uint64_t q, uint64_t n) {
  uint64_t g = 0;
  for (uint64_t x = 2; x < q && !g; ++x) {
    const uint64_t c = host_powmod(x, (q - 1) / (2 * n), q);
    if (host_powmod(c, n, q) == q - 1) g = c;
  }
  const uint64_t g2 = host_mulmod(g, g, q);
  uint64_t cur = g, best = g;
  for (uint64_t e = 0; e < n; ++e) {
    best = std::min(best, cur);
    cur = host_mulmod(cur, g2, q);
  }
  return best;
}

uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// -q^-1 mod 2^64 by Newton's iteration (q odd).
uint64_t mont_neg_inv(uint64_t q) {
  uint64_t x = q;  // correct to 3 bits
  for (int i = 0; i < 6; ++i) x *= 2 - q * x;
  return ~x + 1;
}

size_t align_words(size_t w) { return (w + 31) & ~(size_t)31; }

// Balanced base-256 digits of v < 2^60: v = sum_b d_b 256^b with d_b in
// [-128, 127] for b < 7 and 0 <= d_7 < 18. Adding 128 to each of the seven
// low bytes turns them into the unsigned bytes of z = v + 0x0080...80, whose
// carries propagate exactly as in the digit recurrence.
void balanced_digits(uint64_t v, int8_t d[8]) {
  const uint64_t z = v + 0x0080808080808080ull;
  for (int b = 0; b < 7; ++b) d[b] = (int8_t)((int)((z >> (8 * b)) & 0xFF) - 128);
  d[7] = (int8_t)(z >> 56);
}

// Row rho of a 32-row MFMA tile holds byte b of target tau of the group
// (see k_modup_cols_mx): rho = 8*g8 + 4*hh + e with tau = 2*hh + g8/2 and
// b = 4*(g8%2) + e, so that accumulator i of a lane in half hh of the
// wavefront holds byte i%8 of target 2*hh + i/8.
void row_target_byte(int rho, int& tau, int& b) {
  const int g8 = rho >> 3, hh = (rho >> 2) & 1, e = rho & 3;
  tau = 2 * hh + (g8 >> 1);
  b = 4 * (g8 & 1) + e;
}

// 16 constant bytes of lane l, MFMA step m, for sources 4m + 2*(l/32) + w
// (w = 0, 1; source index s in [0, nsrc)) and row l%32. cst(s, tau) returns
// the BConv constant c_{s,t} and its modulus (modulus 0 = no such target).
template <class Cst>
void mx_lane(uint64_t* out, int l, int m, int nsrc, Cst cst) {
  int tau, b;
  row_target_byte(l & 31, tau, b);
  for (int w = 0; w < 2; ++w) {
    const int s = 4 * m + 2 * (l >> 5) + w;
    uint64_t word = 0;
    uint64_t c = 0, mod = 0;
    if (s < nsrc) cst(s, tau, c, mod);
    if (mod) {
      // byte a of the word: digit b of [c * 256^a]_mod
      uint64_t ca = c;
      for (int a = 0; a < 8; ++a) {
        int8_t dg[8];
        balanced_digits(ca, dg);
        word |= (uint64_t)(uint8_t)dg[b] << (8 * a);
        ca = host_mulmod(ca, 256, mod);
      }
    }
    out[w] = word;
  }
}

}  // namespace

uint64_t host_shoup(uint64_t w, uint64_t q) { return shoup(w, q); }
uint64_t host_mont_neg_inv(uint64_t q) { return mont_neg_inv(q); }

bool derive_params(int dnum, int log_n, int ell, HostParams& hp) {
  if (log_n < 3 || log_n > 17 || ell < 1 || dnum < 1 || dnum > ell) return false;
  hp = HostParams{};
  hp.dnum = dnum;
  hp.log_n = log_n;
  hp.ell = ell;
  hp.n = (size_t)1 << log_n;
  hp.alpha = (ell + dnum - 1) / dnum;
  hp.k = hp.alpha;
  hp.ndig = (ell + hp.alpha - 1) / hp.alpha;
  hp.nl = ell + hp.k;
  const uint64_t step = 2 * (uint64_t)hp.n;
  if (!largest_primes(50, step, ell, hp.mod)) return false;
  if (!largest_primes(60, step, hp.k, hp.mod)) return false;
  for (uint64_t q : hp.mod) hp.psi.push_back(smallest_root(q, hp.n));
  hp.key_ell = ell;
  return true;
}

bool level_params(const HostParams& top, int level, HostParams& hp) {
  if (level < 1 || level > top.ell) return false;
  hp = top;
  hp.ell = level;
  hp.ndig = (level + hp.alpha - 1) / hp.alpha;
  hp.nl = level + hp.k;
  hp.mod.assign(top.mod.begin(), top.mod.begin() + level);
  hp.mod.insert(hp.mod.end(), top.mod.begin() + top.ell, top.mod.end());
  hp.psi.assign(top.psi.begin(), top.psi.begin() + level);
  hp.psi.insert(hp.psi.end(), top.psi.begin() + top.ell, top.psi.end());
  hp.key_ell = top.key_ell;
  return true;
}

void build_tables(const HostParams& hp, std::vector<uint64_t>& blob, DevTables& tb) {
  const size_t n = hp.n;
  const int nl = hp.nl, ell = hp.ell, k = hp.k;
  size_t off = 0;
  auto take = [&](size_t words) {
    const size_t o = off;
    off = align_words(off + words);
    return o;
  };
  const size_t o_limb = take((size_t)nl * (sizeof(LimbC) / 8));
  const size_t o_twf = take((size_t)nl * n * 2);
  const size_t o_twi = take((size_t)nl * n * 2);
  const size_t o_up_pre = take((size_t)ell * 2);
  const size_t o_up_mat = take((size_t)ell * nl * 2);
  const size_t o_dn_pre = take((size_t)k * 2);
  const size_t o_dn_mat = take((size_t)k * ell * 2);
  const size_t o_dn_pinv = take((size_t)ell * 2);
  const size_t o_up_hinv = take((size_t)ell * 2);
  const size_t o_dn_hinv = take((size_t)k * 2);
  const size_t o_twf_d = take((size_t)ell * n);
  const size_t o_twi_d = take((size_t)ell * n);
  const size_t o_up_pre_d = take((size_t)ell);
  const size_t o_up_mat_d = take((size_t)ell * ell);
  const size_t o_dn_mat_d = take((size_t)k * ell * 2);
  const size_t o_dn_pinv_d = take((size_t)ell);
  // MFMA BConv groups: per digit, the Q targets outside the digit in groups
  // of four, then the P targets in groups of four.
  const int alpha = hp.alpha, ndig = hp.ndig;
  const int npg = (k + 3) / 4;
  int up_ng = 0;
  for (int j = 0; j < ndig; ++j) {
    const int na = std::min(alpha, ell - j * alpha);
    up_ng = std::max(up_ng, (ell - na + 3) / 4 + npg);
  }
  const int up_nm = (alpha + 3) / 4, dn_ng = (ell + 3) / 4, dn_nm = (k + 3) / 4;
  const size_t o_up_mx = take((size_t)ndig * up_ng * up_nm * 128);
  const size_t o_dn_mx = take((size_t)dn_ng * dn_nm * 128);
  blob.assign(off, 0);
  // balanced representative of a residue as a double (Q primes only)
  auto bal = [](uint64_t v, uint64_t q) {
    const double d = v <= q / 2 ? (double)v : -(double)(q - v);
    uint64_t bits;
    std::memcpy(&bits, &d, sizeof(bits));
    return bits;
  };

  auto put = [&](size_t o, uint64_t w, uint64_t q) {
    blob[o] = w;
    blob[o + 1] = shoup(w, q);
  };

  for (int t = 0; t < nl; ++t) {
    const uint64_t q = hp.mod[t];
    LimbC L{};
    L.q = q;
    L.two_q = 2 * q;
    L.mont_ninv = mont_neg_inv(q);
    const uint64_t r1 = (uint64_t)(((u128)1 << 64) % q);
    L.r2 = host_mulmod(r1, r1, q);
    L.ninv = inv_prime(n % q, q);
    L.ninv_s = shoup(L.ninv, q);
    L.red_s = shoup(1, q);
    L.r64 = (uint64_t)(((u128)1 << 64) % q);
    L.r64_s = shoup(L.r64, q);
    L.r32 = ((uint64_t)1 << 32) % q;
    L.r32_s = shoup(L.r32, q);
    {
      uint64_t b = bal(L.r32, q);
      std::memcpy(&L.r32_d, &b, sizeof(b));
    }
    // -(2^51 + 2^83) mod q
    const uint64_t c51 = ((uint64_t)1 << 51) % q;
    const uint64_t c83 = (uint64_t)(((u128)1 << 83) % q);
    L.cadj = (2 * q - c51 - c83) % q;
    L.qd = (double)q;
    L.qinv = 1.0 / (double)q;
    {
      uint64_t b = bal(L.ninv, q);
      std::memcpy(&L.ninv_d, &b, sizeof(b));
    }
    std::copy_n(reinterpret_cast<const uint64_t*>(&L), sizeof(LimbC) / 8, blob.begin() + o_limb + (size_t)t * (sizeof(LimbC) / 8));

    // powers psi^e and psi^-e for e < N, then the bit-reversed tables
    std::vector<uint64_t> pw(n), ipw(n);
    const uint64_t psi = hp.psi[t], ipsi = inv_prime(psi, q);
    pw[0] = ipw[0] = 1;
    for (size_t e = 1; e < n; ++e) {
      pw[e] = host_mulmod(pw[e - 1], psi, q);
      ipw[e] = host_mulmod(ipw[e - 1], ipsi, q);
    }
    for (size_t i = 0; i < n; ++i) {
      const uint32_t r = bitrev((uint32_t)i, hp.log_n);
      put(o_twf + ((size_t)t * n + i) * 2, pw[r], q);
      put(o_twi + ((size_t)t * n + i) * 2, ipw[r], q);
      if (t < ell) {
        blob[o_twf_d + (size_t)t * n + i] = bal(pw[r], q);
        blob[o_twi_d + (size_t)t * n + i] = bal(ipw[r], q);
      }
    }
  }

  // ModUp: per source limb i of digit j
  for (int i = 0; i < ell; ++i) {
    const int j = i / hp.alpha;
    const int lo = j * hp.alpha, hi = std::min(lo + hp.alpha, ell);
    const uint64_t qi = hp.mod[i];
    uint64_t hat = 1;
    for (int i2 = lo; i2 < hi; ++i2)
      if (i2 != i) hat = host_mulmod(hat, hp.mod[i2] % qi, qi);
    const uint64_t hinv = inv_prime(hat, qi);
    put(o_up_hinv + (size_t)i * 2, hinv, qi);
    const uint64_t pre = host_mulmod(hinv, inv_prime(n % qi, qi), qi);
    put(o_up_pre + (size_t)i * 2, pre, qi);
    blob[o_up_pre_d + i] = bal(pre, qi);
    for (int t = 0; t < nl; ++t) {
      const uint64_t m = hp.mod[t];
      uint64_t v = 1;
      for (int i2 = lo; i2 < hi; ++i2)
        if (i2 != i) v = host_mulmod(v, hp.mod[i2] % m, m);
      put(o_up_mat + ((size_t)i * nl + t) * 2, v, m);
      if (t < ell) blob[o_up_mat_d + (size_t)i * ell + t] = bal(v, m);
    }
  }

  // ModDown
  for (int m = 0; m < k; ++m) {
    const uint64_t pm = hp.mod[ell + m];
    uint64_t hat = 1;
    for (int m2 = 0; m2 < k; ++m2)
      if (m2 != m) hat = host_mulmod(hat, hp.mod[ell + m2] % pm, pm);
    const uint64_t hinv = inv_prime(hat, pm);
    put(o_dn_hinv + (size_t)m * 2, hinv, pm);
    put(o_dn_pre + (size_t)m * 2, host_mulmod(hinv, inv_prime(n % pm, pm), pm), pm);
    for (int i = 0; i < ell; ++i) {
      const uint64_t qi = hp.mod[i];
      uint64_t v = 1;
      for (int m2 = 0; m2 < k; ++m2)
        if (m2 != m) v = host_mulmod(v, hp.mod[ell + m2] % qi, qi);
      put(o_dn_mat + ((size_t)m * ell + i) * 2, v, qi);
      blob[o_dn_mat_d + ((size_t)m * ell + i) * 2] = bal(host_mulmod(v, (1ull << 30) % qi, qi), qi);
      blob[o_dn_mat_d + ((size_t)m * ell + i) * 2 + 1] = bal(v, qi);
    }
  }
  for (int i = 0; i < ell; ++i) {
    const uint64_t qi = hp.mod[i];
    uint64_t pmod = 1;
    for (int m = 0; m < k; ++m) pmod = host_mulmod(pmod, hp.mod[ell + m] % qi, qi);
    const uint64_t pinv = inv_prime(pmod, qi);
    put(o_dn_pinv + (size_t)i * 2, pinv, qi);
    blob[o_dn_pinv_d + i] = bal(pinv, qi);
  }

  // MFMA BConv constant operands
  for (int j = 0; j < ndig; ++j) {
    const int lo = j * alpha, na = std::min(alpha, ell - lo);
    const int nq = ell - na, nqg = (nq + 3) / 4;
    for (int g = 0; g < nqg + npg; ++g)
      for (int m = 0; m < up_nm; ++m)
        for (int l = 0; l < 64; ++l) {
          uint64_t* dst = &blob[o_up_mx + ((((size_t)j * up_ng + g) * up_nm + m) * 64 + l) * 2];
          mx_lane(dst, l, m, na, [&](int sidx, int tau, uint64_t& c, uint64_t& mod) {
            int t = -1;
            if (g < nqg) {
              const int u = 4 * g + tau;
              if (u < nq) t = u < lo ? u : u + na;
            } else {
              const int v = 4 * (g - nqg) + tau;
              if (v < k) t = ell + v;
            }
            if (t < 0) return;
            c = blob[o_up_mat + ((size_t)(lo + sidx) * nl + t) * 2];
            mod = hp.mod[t];
          });
        }
  }
  for (int g = 0; g < dn_ng; ++g)
    for (int m = 0; m < dn_nm; ++m)
      for (int l = 0; l < 64; ++l) {
        uint64_t* dst = &blob[o_dn_mx + (((size_t)g * dn_nm + m) * 64 + l) * 2];
        mx_lane(dst, l, m, k, [&](int sidx, int tau, uint64_t& c, uint64_t& mod) {
          const int t = 4 * g + tau;
          if (t >= ell) return;
          c = blob[o_dn_mat + ((size_t)sidx * ell + t) * 2];
          mod = hp.mod[t];
        });
      }

  tb.log_n = hp.log_n;
  tb.ell = ell;
  tb.k = k;
  tb.nl = nl;
  tb.alpha = hp.alpha;
  tb.ndig = hp.ndig;
  auto at = [](size_t o) { return reinterpret_cast<const uint64_t*>(o * sizeof(uint64_t)); };
  tb.limb = reinterpret_cast<const LimbC*>(at(o_limb));
  tb.twf = at(o_twf);
  tb.twi = at(o_twi);
  tb.up_pre = at(o_up_pre);
  tb.up_mat = at(o_up_mat);
  tb.dn_pre = at(o_dn_pre);
  tb.dn_mat = at(o_dn_mat);
  tb.dn_pinv = at(o_dn_pinv);
  tb.up_hinv = at(o_up_hinv);
  tb.dn_hinv = at(o_dn_hinv);
  tb.up_mx = at(o_up_mx);
  tb.dn_mx = at(o_dn_mx);
  tb.up_ng = up_ng;
  tb.up_nm = up_nm;
  tb.dn_ng = dn_ng;
  tb.dn_nm = dn_nm;
  tb.evk_nl = hp.key_ell + k;
  tb.evk_p0 = hp.key_ell;
  auto atd = [](size_t o) { return reinterpret_cast<const double*>(o * sizeof(uint64_t)); };
  tb.twf_d = atd(o_twf_d);
  tb.twi_d = atd(o_twi_d);
  tb.up_pre_d = atd(o_up_pre_d);
  tb.up_mat_d = atd(o_up_mat_d);
  tb.dn_mat_d = atd(o_dn_mat_d);
  tb.dn_pinv_d = atd(o_dn_pinv_d);
}

}  // namespace ks
