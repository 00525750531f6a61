/*
 * Plain CPU oracle of the CKKS hybrid KeySwitch (test infrastructure).
 *
 * This file is test infrastructure. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it. It shares no code with the
 * GPU library: every modular product here is a 128-bit product reduced with
 * `%`, every transform is the textbook radix-2 loop, and every base
 * conversion is the defining sum. Nothing is blocked, fused or reordered.
 *
 * What it follows (Background, "KeySwitch" subsection, and Fig. 1 of the
 * paper): the input polynomial d (a ciphertext component over the Q basis, in
 * NTT form) is split into digits; each digit is raised to the basis PQ by
 * iNTT -> BConv -> NTT (ModUp), multiplied by the evaluation key of its digit
 * and summed over digits (KeyMult), and the sum is brought back to Q by
 * iNTT -> BConv -> NTT followed by the subtraction and the division by P
 * (ModDown). The paper leaves the following choices open; the oracle fixes
 * them as stated next to each function:
 *   - the ring is Z_Q[x]/(x^N + 1) (negacyclic);
 *   - Q holds `ell` primes q < 2^50 and P holds k = alpha primes p < 2^60,
 *     all = 1 (mod 2N), the largest such primes in descending order;
 *   - alpha = ceil(ell / dnum), digit j holds Q limbs [j*alpha, min((j+1)*alpha, ell));
 *   - psi is the smallest primitive 2N-th root of unity mod each prime;
 *   - NTT(a)[t] = sum_i a_i psi^(i*(2*brv(t)+1)) (bit-reversed evaluation order);
 *   - BConv is the fast (uncorrected) conversion with y_i in [0, q_i);
 *   - ModDown ends with (acc_Q - conv) * P^-1, without a rounding offset;
 *   - at a level l < ell (a ciphertext that has lost its last ell - l
 *     limbs), the KeySwitch keeps the top level's P and alpha, works over
 *     q_0..q_{l-1}, uses the digits D_j restricted to those limbs
 *     (ceil(l / alpha) of them) and the top-level key restricted to the limbs
 *     of q_0..q_{l-1} and P (the `_level` entry points).
 *
 * Layouts (all uint64, canonical residues, coefficient index fastest):
 *   d   [batch][ell][N]              over q_0..q_{ell-1}, NTT form
 *   ext [batch][ndig][ell+k][N]      over q_0..q_{ell-1}, p_0..p_{k-1}, NTT form
 *   evk [ndig][2][ell+k][N]          component 0 = b, 1 = a, NTT form
 *   acc [batch][2][ell+k][N]         NTT form
 *   out [batch][2][ell][N]           NTT form
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef unsigned __int128 u128;

#define ORC_MAX_LIMBS 160

/* ---------------------------------------------------------------- scalar */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a * b) % m);
}
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a + b) % m);
}
static uint64_t submod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a + m - b) % m);
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}
/* Inverse modulo a prime, by Fermat's little theorem. */
static uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }

/* Deterministic Miller-Rabin; the first twelve primes as bases decide every
 * n < 3.3e24 (Sorenson and Webster, 2015). */
static int is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

static uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* SplitMix64 (Steele, Lea and Flood, 2014) in counter form: draw number
 * `idx` (0-based) of the stream with seed `seed`. */
static uint64_t splitmix64(uint64_t seed, uint64_t idx) {
  uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------ parameters */

typedef struct {
  int dnum, log_n, ell, k, alpha, ndig;
  size_t n;
  uint64_t mod[ORC_MAX_LIMBS]; /* q_0..q_{ell-1}, p_0..p_{k-1} */
  uint64_t psi[ORC_MAX_LIMBS];
} orc_params;

/* The `count` largest primes below 2^bits that are = 1 (mod 2N), descending. */
static int gen_primes(int bits, uint64_t two_n, int count, uint64_t* out) {
  uint64_t top = (bits == 64) ? ~0ull : ((1ull << bits) - 1);
  uint64_t c = (top / two_n) * two_n + 1;
  if (c > top) c -= two_n;
  int got = 0;
  while (got < count) {
    if (c <= two_n) return -1;
    if (is_prime(c)) out[got++] = c;
    c -= two_n;
  }
  return 0;
}

/* The smallest primitive 2N-th root of unity mod q. A primitive one is
 * g = x^((q-1)/2N) with g^N = -1; all of them are the odd powers of g. */
static uint64_t find_psi(uint64_t q, size_t n) {
  uint64_t g = 0;
  for (uint64_t x = 2; x < q; ++x) {
    uint64_t c = powmod(x, (q - 1) / (2 * n), q);
    if (powmod(c, n, q) == q - 1) { g = c; break; }
  }
  uint64_t g2 = mulmod(g, g, q), cur = g, best = g;
  for (size_t j = 0; j < n; ++j) {
    if (cur < best) best = cur;
    cur = mulmod(cur, g2, q);
  }
  return best;
}

static int derive(int dnum, int log_n, int ell, orc_params* p) {
  if (log_n < 1 || log_n > 20 || ell < 1 || dnum < 1 || dnum > ell) return -1;
  memset(p, 0, sizeof(*p));
  p->dnum = dnum;
  p->log_n = log_n;
  p->ell = ell;
  p->n = (size_t)1 << log_n;
  p->alpha = (ell + dnum - 1) / dnum;
  p->k = p->alpha;
  p->ndig = (ell + p->alpha - 1) / p->alpha;
  if (ell + p->k > ORC_MAX_LIMBS) return -1;
  uint64_t two_n = 2 * (uint64_t)p->n;
  if (gen_primes(50, two_n, ell, p->mod) != 0) return -1;
  if (gen_primes(60, two_n, p->k, p->mod + ell) != 0) return -1;
  for (int t = 0; t < ell + p->k; ++t) p->psi[t] = find_psi(p->mod[t], p->n);
  return 0;
}

static int digit_lo(const orc_params* p, int j) { return j * p->alpha; }
static int digit_hi(const orc_params* p, int j) {
  int h = (j + 1) * p->alpha;
  return h < p->ell ? h : p->ell;
}

/* Parameters of level `level` of the (dnum, N, ell) set: Q shrinks to its
 * first `level` primes, P, k and alpha stay, the digits are those of the
 * top level cut at `level`. */
static int derive_level(int dnum, int log_n, int ell, int level, orc_params* p) {
  if (derive(dnum, log_n, ell, p) != 0 || level < 1 || level > ell) return -1;
  for (int m = 0; m < p->k; ++m) {
    p->mod[level + m] = p->mod[ell + m];
    p->psi[level + m] = p->psi[ell + m];
  }
  p->ell = level;
  p->ndig = (level + p->alpha - 1) / p->alpha;
  return 0;
}

/* The top-level key [ndig_top][2][ell+k][N] restricted to the limbs of level
 * p->ell: [p->ndig][2][p->ell+k][N] (newly allocated). */
static uint64_t* key_at_level(const orc_params* p, int ell_top, const uint64_t* evk) {
  size_t n = p->n;
  int nl = p->ell + p->k, nlt = ell_top + p->k;
  uint64_t* key = (uint64_t*)malloc((size_t)p->ndig * 2 * nl * n * sizeof(uint64_t));
  if (!key) return NULL;
  for (int j = 0; j < p->ndig; ++j)
    for (int c = 0; c < 2; ++c)
      for (int t = 0; t < nl; ++t) {
        int row = t < p->ell ? t : ell_top + (t - p->ell);
        memcpy(key + (((size_t)j * 2 + c) * nl + t) * n, evk + (((size_t)j * 2 + c) * nlt + row) * n,
               n * sizeof(uint64_t));
      }
  return key;
}

/* ------------------------------------------------------------------ NTT */

/* Forward negacyclic NTT, in place, textbook iterative Cooley-Tukey with the
 * powers psi^brv(m+i): output slot t holds sum_i a_i psi^(i*(2*brv(t)+1)). */
static void ntt_limb(uint64_t q, uint64_t psi, int log_n, uint64_t* a) {
  size_t n = (size_t)1 << log_n;
  uint64_t* pw = (uint64_t*)malloc(n * sizeof(uint64_t));
  pw[0] = 1;
  for (size_t e = 1; e < n; ++e) pw[e] = mulmod(pw[e - 1], psi, q);
  for (size_t m = 1, t = n / 2; m < n; m *= 2, t /= 2) {
    for (size_t i = 0; i < m; ++i) {
      uint64_t w = pw[brv((uint32_t)(m + i), log_n)];
      for (size_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        uint64_t u = a[j], v = mulmod(a[j + t], w, q);
        a[j] = addmod(u, v, q);
        a[j + t] = submod(u, v, q);
      }
    }
  }
  free(pw);
}

/* Inverse of ntt_limb: Gentleman-Sande loop with psi^-brv(m+i), then N^-1. */
static void intt_limb(uint64_t q, uint64_t psi, int log_n, uint64_t* a) {
  size_t n = (size_t)1 << log_n;
  uint64_t psi_inv = invmod(psi, q);
  uint64_t* pw = (uint64_t*)malloc(n * sizeof(uint64_t));
  pw[0] = 1;
  for (size_t e = 1; e < n; ++e) pw[e] = mulmod(pw[e - 1], psi_inv, q);
  for (size_t m = n / 2, t = 1; m >= 1; m /= 2, t *= 2) {
    for (size_t i = 0; i < m; ++i) {
      uint64_t w = pw[brv((uint32_t)(m + i), log_n)];
      for (size_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        uint64_t u = a[j], v = a[j + t];
        a[j] = addmod(u, v, q);
        a[j + t] = mulmod(submod(u, v, q), w, q);
      }
    }
  }
  uint64_t n_inv = invmod((uint64_t)(n % q), q);
  for (size_t j = 0; j < n; ++j) a[j] = mulmod(a[j], n_inv, q);
  free(pw);
}

/* ----------------------------------------------------------------- BConv */

/* Fast base conversion from the source primes src[0..ns-1] to the target
 * primes dst[0..nd-1] (BConv in the KeySwitch description):
 *   y_i = x_i * [(S/s_i)^-1]_{s_i} mod s_i,
 *   z_t = sum_i y_i * [S/s_i]_t mod t,  S = prod_i s_i.
 * x: [ns][N] coefficient form, z: [nd][N] coefficient form. */
static void bconv_core(const uint64_t* src, int ns, const uint64_t* dst_mod, int nd,
                       size_t n, const uint64_t* x, uint64_t* z) {
  uint64_t hat_inv[ORC_MAX_LIMBS];
  for (int i = 0; i < ns; ++i) {
    uint64_t prod = 1;
    for (int i2 = 0; i2 < ns; ++i2)
      if (i2 != i) prod = mulmod(prod, src[i2] % src[i], src[i]);
    hat_inv[i] = invmod(prod, src[i]);
  }
  uint64_t* y = (uint64_t*)malloc((size_t)ns * n * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
  for (int i = 0; i < ns; ++i)
    for (size_t c = 0; c < n; ++c) y[(size_t)i * n + c] = mulmod(x[(size_t)i * n + c], hat_inv[i], src[i]);
#pragma omp parallel for schedule(static)
  for (int t = 0; t < nd; ++t) {
    uint64_t tm = dst_mod[t];
    uint64_t hat[ORC_MAX_LIMBS];
    for (int i = 0; i < ns; ++i) {
      uint64_t prod = 1;
      for (int i2 = 0; i2 < ns; ++i2)
        if (i2 != i) prod = mulmod(prod, src[i2] % tm, tm);
      hat[i] = prod;
    }
    for (size_t c = 0; c < n; ++c) {
      uint64_t s = 0;
      for (int i = 0; i < ns; ++i) s = addmod(s, mulmod(y[(size_t)i * n + c] % tm, hat[i], tm), tm);
      z[(size_t)t * n + c] = s;
    }
  }
  free(y);
}

/* ---------------------------------------------------------------- phases */

/* ModUp of one ciphertext component: ext[j][t] for every digit j and limb t
 * of PQ. On the digit's own limbs the input residue is kept; elsewhere
 * ext = NTT_t(BConv_{D_j -> t}(INTT(d restricted to D_j))). */
static void modup_one(const orc_params* p, const uint64_t* d, uint64_t* ext) {
  size_t n = p->n;
  int nl = p->ell + p->k;
  for (int j = 0; j < p->ndig; ++j) {
    int lo = digit_lo(p, j), hi = digit_hi(p, j), na = hi - lo;
    uint64_t* x = (uint64_t*)malloc((size_t)na * n * sizeof(uint64_t));
    memcpy(x, d + (size_t)lo * n, (size_t)na * n * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < na; ++i) intt_limb(p->mod[lo + i], p->psi[lo + i], p->log_n, x + (size_t)i * n);
    uint64_t dst_mod[ORC_MAX_LIMBS];
    int dst_idx[ORC_MAX_LIMBS], nd = 0;
    for (int t = 0; t < nl; ++t)
      if (t < lo || t >= hi) { dst_mod[nd] = p->mod[t]; dst_idx[nd] = t; ++nd; }
    uint64_t* z = (uint64_t*)malloc((size_t)nd * n * sizeof(uint64_t));
    bconv_core(p->mod + lo, na, dst_mod, nd, n, x, z);
    uint64_t* e = ext + (size_t)j * nl * n;
#pragma omp parallel for schedule(static)
    for (int u = 0; u < nd; ++u) {
      int t = dst_idx[u];
      memcpy(e + (size_t)t * n, z + (size_t)u * n, n * sizeof(uint64_t));
      ntt_limb(p->mod[t], p->psi[t], p->log_n, e + (size_t)t * n);
    }
    for (int t = lo; t < hi; ++t) memcpy(e + (size_t)t * n, d + (size_t)t * n, n * sizeof(uint64_t));
    free(x);
    free(z);
  }
}

/* KeyMult: acc[c][t] = sum_j ext[j][t] * evk[j][c][t] mod t, c in {0, 1}. */
static void keymult_one(const orc_params* p, const uint64_t* ext, const uint64_t* evk, uint64_t* acc) {
  size_t n = p->n;
  int nl = p->ell + p->k;
#pragma omp parallel for schedule(static)
  for (int ct = 0; ct < 2 * nl; ++ct) {
    int c = ct / nl, t = ct % nl;
    uint64_t m = p->mod[t];
    for (size_t x = 0; x < n; ++x) {
      uint64_t s = 0;
      for (int j = 0; j < p->ndig; ++j)
        s = addmod(s, mulmod(ext[((size_t)j * nl + t) * n + x], evk[(((size_t)j * 2 + c) * nl + t) * n + x], m), m);
      acc[((size_t)c * nl + t) * n + x] = s;
    }
  }
}

/* ModDown: out[c][i] = (acc[c][q_i] - NTT(BConv_{P -> q_i}(INTT(acc[c][P])))) * P^-1 mod q_i. */
static void moddown_one(const orc_params* p, const uint64_t* acc, uint64_t* out) {
  size_t n = p->n;
  int nl = p->ell + p->k, ell = p->ell, k = p->k;
  uint64_t* x = (uint64_t*)malloc((size_t)k * n * sizeof(uint64_t));
  uint64_t* z = (uint64_t*)malloc((size_t)ell * n * sizeof(uint64_t));
  for (int c = 0; c < 2; ++c) {
    const uint64_t* a = acc + (size_t)c * nl * n;
    memcpy(x, a + (size_t)ell * n, (size_t)k * n * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int m = 0; m < k; ++m) intt_limb(p->mod[ell + m], p->psi[ell + m], p->log_n, x + (size_t)m * n);
    bconv_core(p->mod + ell, k, p->mod, ell, n, x, z);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < ell; ++i) {
      uint64_t q = p->mod[i];
      uint64_t pmod = 1;
      for (int m = 0; m < k; ++m) pmod = mulmod(pmod, p->mod[ell + m] % q, q);
      uint64_t p_inv = invmod(pmod, q);
      uint64_t* zi = z + (size_t)i * n;
      ntt_limb(q, p->psi[i], p->log_n, zi);
      for (size_t t = 0; t < n; ++t)
        out[((size_t)c * ell + i) * n + t] = mulmod(submod(a[(size_t)i * n + t], zi[t], q), p_inv, q);
    }
  }
  free(x);
  free(z);
}

/* ------------------------------------------------------------------ ABI */

int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/* Parameter derivation. moduli and psi receive ell + k values; info receives
 * {n, ell, k, alpha, ndig}. */
int orc_derive(int dnum, int log_n, int ell, uint64_t* moduli, uint64_t* psi, int64_t* info) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  for (int t = 0; t < ell + p.k; ++t) { moduli[t] = p.mod[t]; psi[t] = p.psi[t]; }
  info[0] = (int64_t)p.n; info[1] = p.ell; info[2] = p.k; info[3] = p.alpha; info[4] = p.ndig;
  return 0;
}

int orc_is_prime(uint64_t n) { return is_prime(n); }

/* In-place transforms of `count` consecutive limbs of N values, modulus q and
 * root psi shared by all of them. */
void orc_ntt(uint64_t q, uint64_t psi, int log_n, uint64_t* a, int count) {
  size_t n = (size_t)1 << log_n;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < count; ++c) ntt_limb(q, psi, log_n, a + (size_t)c * n);
}
void orc_intt(uint64_t q, uint64_t psi, int log_n, uint64_t* a, int count) {
  size_t n = (size_t)1 << log_n;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < count; ++c) intt_limb(q, psi, log_n, a + (size_t)c * n);
}

/* BConv in coefficient form. src_set = digit index j (source D_j, target
 * PQ minus D_j in basis order) or -1 (source P, target Q).
 * src [batch][|source|][N], dst [batch][|target|][N]. */
int orc_bconv(int dnum, int log_n, int ell, int src_set, const uint64_t* src, uint64_t* dst, int batch) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  int nl = p.ell + p.k;
  uint64_t src_mod[ORC_MAX_LIMBS], dst_mod[ORC_MAX_LIMBS];
  int ns = 0, nd = 0;
  if (src_set < 0) {
    for (int m = 0; m < p.k; ++m) src_mod[ns++] = p.mod[p.ell + m];
    for (int i = 0; i < p.ell; ++i) dst_mod[nd++] = p.mod[i];
  } else {
    if (src_set >= p.ndig) return -1;
    int lo = digit_lo(&p, src_set), hi = digit_hi(&p, src_set);
    for (int t = 0; t < nl; ++t) {
      if (t >= lo && t < hi) src_mod[ns++] = p.mod[t];
      else dst_mod[nd++] = p.mod[t];
    }
  }
  for (int b = 0; b < batch; ++b)
    bconv_core(src_mod, ns, dst_mod, nd, p.n, src + (size_t)b * ns * p.n, dst + (size_t)b * nd * p.n);
  return 0;
}

int orc_modup(int dnum, int log_n, int ell, const uint64_t* d, uint64_t* ext, int batch) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  size_t dsz = (size_t)p.ell * p.n, esz = (size_t)p.ndig * (p.ell + p.k) * p.n;
  for (int b = 0; b < batch; ++b) modup_one(&p, d + b * dsz, ext + b * esz);
  return 0;
}

int orc_keymult(int dnum, int log_n, int ell, const uint64_t* ext, const uint64_t* evk, uint64_t* acc, int batch) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  size_t esz = (size_t)p.ndig * (p.ell + p.k) * p.n, asz = (size_t)2 * (p.ell + p.k) * p.n;
  for (int b = 0; b < batch; ++b) keymult_one(&p, ext + b * esz, evk, acc + b * asz);
  return 0;
}

int orc_moddown(int dnum, int log_n, int ell, const uint64_t* acc, uint64_t* out, int batch) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  size_t asz = (size_t)2 * (p.ell + p.k) * p.n, osz = (size_t)2 * p.ell * p.n;
  for (int b = 0; b < batch; ++b) moddown_one(&p, acc + b * asz, out + b * osz);
  return 0;
}

/* The whole KeySwitch: ModUp, KeyMult, ModDown, one ciphertext at a time. */
int orc_keyswitch(int dnum, int log_n, int ell, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  size_t nl = (size_t)(p.ell + p.k);
  size_t dsz = (size_t)p.ell * p.n, osz = (size_t)2 * p.ell * p.n;
  uint64_t* ext = (uint64_t*)malloc((size_t)p.ndig * nl * p.n * sizeof(uint64_t));
  uint64_t* acc = (uint64_t*)malloc(2 * nl * p.n * sizeof(uint64_t));
  if (!ext || !acc) { free(ext); free(acc); return -2; }
  for (int b = 0; b < batch; ++b) {
    modup_one(&p, d + b * dsz, ext);
    keymult_one(&p, ext, evk, acc);
    moddown_one(&p, acc, out + b * osz);
  }
  free(ext);
  free(acc);
  return 0;
}

/* The same steps at level `level` (1 <= level <= ell), with the key of the
 * top level: d [batch][level][N], ext [batch][ceil(level/alpha)][level+k][N],
 * evk [ndig_top][2][ell+k][N], acc [batch][2][level+k][N],
 * out [batch][2][level][N]. level = ell gives the top-level functions. */
int orc_modup_level(int dnum, int log_n, int ell, int level, const uint64_t* d, uint64_t* ext, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  size_t dsz = (size_t)p.ell * p.n, esz = (size_t)p.ndig * (p.ell + p.k) * p.n;
  for (int b = 0; b < batch; ++b) modup_one(&p, d + b * dsz, ext + b * esz);
  return 0;
}

int orc_keymult_level(int dnum, int log_n, int ell, int level, const uint64_t* ext, const uint64_t* evk,
                      uint64_t* acc, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  uint64_t* key = key_at_level(&p, ell, evk);
  if (!key) return -2;
  size_t esz = (size_t)p.ndig * (p.ell + p.k) * p.n, asz = (size_t)2 * (p.ell + p.k) * p.n;
  for (int b = 0; b < batch; ++b) keymult_one(&p, ext + b * esz, key, acc + b * asz);
  free(key);
  return 0;
}

int orc_moddown_level(int dnum, int log_n, int ell, int level, const uint64_t* acc, uint64_t* out, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  size_t asz = (size_t)2 * (p.ell + p.k) * p.n, osz = (size_t)2 * p.ell * p.n;
  for (int b = 0; b < batch; ++b) moddown_one(&p, acc + b * asz, out + b * osz);
  return 0;
}

int orc_keyswitch_level(int dnum, int log_n, int ell, int level, const uint64_t* d, const uint64_t* evk,
                        uint64_t* out, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  size_t nl = (size_t)(p.ell + p.k);
  size_t dsz = (size_t)p.ell * p.n, osz = (size_t)2 * p.ell * p.n;
  uint64_t* key = key_at_level(&p, ell, evk);
  uint64_t* ext = (uint64_t*)malloc((size_t)p.ndig * nl * p.n * sizeof(uint64_t));
  uint64_t* acc = (uint64_t*)malloc(2 * nl * p.n * sizeof(uint64_t));
  if (!key || !ext || !acc) { free(key); free(ext); free(acc); return -2; }
  for (int b = 0; b < batch; ++b) {
    modup_one(&p, d + b * dsz, ext);
    keymult_one(&p, ext, key, acc);
    moddown_one(&p, acc, out + b * osz);
  }
  free(key);
  free(ext);
  free(acc);
  return 0;
}

/* ---------------------------------------------------------------- keygen */

/* Ternary secret with exactly h nonzeros: positions by a partial
 * Fisher-Yates shuffle, signs from the low bit of a second draw. */
static void ternary(uint64_t seed, size_t n, int h, int8_t* s) {
  uint32_t* perm = (uint32_t*)malloc(n * sizeof(uint32_t));
  for (size_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  memset(s, 0, n);
  uint64_t idx = 0;
  for (int i = 0; i < h; ++i) {
    uint64_t r = splitmix64(seed, idx++);
    size_t j = (size_t)i + (size_t)(r % (n - (size_t)i));
    uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    uint64_t r2 = splitmix64(seed, idx++);
    s[perm[i]] = (r2 & 1) ? 1 : -1;
  }
  free(perm);
}

/* Standard deviation of the evaluation-key errors and the cut of their tail
 * (|e| <= 19, i.e. about 6 sigma); the paper does not state a sampler. */
#define ORC_SIGMA 3.2
#define ORC_ERR_CUT 19.0

/* Rounded normal with standard deviation sigma by Box-Muller, rejected
 * beyond the cut. */
static void gaussian(uint64_t seed, size_t count, double sigma, int64_t* e) {
  const double two_pi = 6.283185307179586;
  uint64_t idx = 0;
  for (size_t i = 0; i < count; ++i) {
    for (;;) {
      double u1 = ((double)(splitmix64(seed, idx++) >> 11) + 1.0) * 0x1.0p-53;
      double u2 = (double)(splitmix64(seed, idx++) >> 11) * 0x1.0p-53;
      double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
      double v = nearbyint(sigma * z);
      if (fabs(v) <= ORC_ERR_CUT) { e[i] = (int64_t)v; break; }
    }
  }
}

static uint64_t signed_mod(int64_t v, uint64_t m) {
  return v >= 0 ? (uint64_t)v % m : (m - ((uint64_t)(-v) % m)) % m;
}

/* Evaluation key for switching from secret s_from to secret s_to (both
 * given by their integer coefficients), one pair per digit j:
 *   a_j uniform mod each t (draw (j*(ell+k)+t)*N + x of seed_a),
 *   e_j rounded Gaussian (seed_e, digit after digit),
 *   b_j = -a_j*s_to + e_j + [t in D_j] * [P]_t * s_from   (NTT form, per limb t).
 * With noiseless != 0 every e_j is zero. */
static void make_key(const orc_params* pp, const int64_t* s_from, const int64_t* s_to, uint64_t seed_a,
                     uint64_t seed_e, int noiseless, uint64_t* evk) {
  const orc_params p = *pp;
  size_t n = p.n;
  int nl = p.ell + p.k;
  int64_t* e = (int64_t*)calloc((size_t)p.ndig * n, sizeof(int64_t));
  if (!noiseless) gaussian(seed_e, (size_t)p.ndig * n, ORC_SIGMA, e);
  for (int j = 0; j < p.ndig; ++j) {
    int lo = digit_lo(&p, j), hi = digit_hi(&p, j);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nl; ++t) {
      uint64_t m = p.mod[t];
      uint64_t* sh = (uint64_t*)malloc(n * sizeof(uint64_t));
      uint64_t* s2h = (uint64_t*)malloc(n * sizeof(uint64_t));
      uint64_t* eh = (uint64_t*)malloc(n * sizeof(uint64_t));
      for (size_t x = 0; x < n; ++x) {
        sh[x] = signed_mod(s_from[x], m);
        s2h[x] = signed_mod(s_to[x], m);
        eh[x] = signed_mod(e[(size_t)j * n + x], m);
      }
      ntt_limb(m, p.psi[t], p.log_n, sh);
      ntt_limb(m, p.psi[t], p.log_n, s2h);
      ntt_limb(m, p.psi[t], p.log_n, eh);
      uint64_t pm = 1;
      for (int u = 0; u < p.k; ++u) pm = mulmod(pm, p.mod[p.ell + u] % m, m);
      int own = (t >= lo && t < hi);
      uint64_t* b = evk + (((size_t)j * 2 + 0) * nl + t) * n;
      uint64_t* a = evk + (((size_t)j * 2 + 1) * nl + t) * n;
      for (size_t x = 0; x < n; ++x) {
        a[x] = splitmix64(seed_a, ((size_t)j * nl + t) * n + x) % m;
        uint64_t v = submod(eh[x], mulmod(a[x], s2h[x], m), m);
        if (own) v = addmod(v, mulmod(pm, sh[x], m), m);
        b[x] = v;
      }
      free(sh); free(s2h); free(eh);
    }
  }
  free(e);
}

/* The two samplers on their own, so that tests can check them against their
 * definitions: a ternary secret of n coefficients with exactly h nonzeros,
 * and `count` rounded-Gaussian errors of standard deviation sigma (the keys
 * use ORC_SIGMA). */
int orc_sample_ternary(uint64_t seed, int64_t n, int h, int8_t* s) {
  if (n <= 0 || h < 0 || (int64_t)h > n) return -1;
  ternary(seed, (size_t)n, h, s);
  return 0;
}

int orc_sample_gaussian(uint64_t seed, int64_t count, double sigma, int64_t* e) {
  if (count < 0 || !(sigma > 0.0)) return -1;
  gaussian(seed, (size_t)count, sigma, e);
  return 0;
}

double orc_key_sigma(void) { return ORC_SIGMA; }

/* The key from s to s2 for two fresh ternary secrets with h nonzeros each
 * (seeds seed_s, seed_s2); s_out and s2_out receive them. */
int orc_keygen(int dnum, int log_n, int ell, int h, uint64_t seed_s, uint64_t seed_s2, uint64_t seed_a,
               uint64_t seed_e, int noiseless, int8_t* s_out, int8_t* s2_out, uint64_t* evk) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  size_t n = p.n;
  if (h < 0 || (size_t)h > n) return -1;
  ternary(seed_s, n, h, s_out);
  ternary(seed_s2, n, h, s2_out);
  int64_t* a = (int64_t*)malloc(n * sizeof(int64_t));
  int64_t* b = (int64_t*)malloc(n * sizeof(int64_t));
  for (size_t x = 0; x < n; ++x) { a[x] = s_out[x]; b[x] = s2_out[x]; }
  make_key(&p, a, b, seed_a, seed_e, noiseless, evk);
  free(a);
  free(b);
  return 0;
}

/* The key from an arbitrary s_from (for instance s*s for relinearisation,
 * or an automorphism of s for rotation) to s_to. */
int orc_keygen_pair(int dnum, int log_n, int ell, const int64_t* s_from, const int64_t* s_to, uint64_t seed_a,
                    uint64_t seed_e, int noiseless, uint64_t* evk) {
  orc_params p;
  if (derive(dnum, log_n, ell, &p) != 0) return -1;
  make_key(&p, s_from, s_to, seed_a, seed_e, noiseless, evk);
  return 0;
}

/* ------------------------------------------------- HMUL and HROT (test side) */

/* The Galois automorphism a(X) -> a(X^g) (g odd) of `count` limbs in NTT form,
 * computed in the coefficient domain: coefficient i moves to i*g mod 2N,
 * negated when that lands in [N, 2N) (X^N = -1). */
void orc_automorph(uint64_t q, uint64_t psi, int log_n, const uint64_t* a, uint64_t g, uint64_t* out, int count) {
  size_t n = (size_t)1 << log_n;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < count; ++c) {
    uint64_t* x = (uint64_t*)malloc(n * sizeof(uint64_t));
    memcpy(x, a + (size_t)c * n, n * sizeof(uint64_t));
    intt_limb(q, psi, log_n, x);
    uint64_t* y = out + (size_t)c * n;
    for (size_t i = 0; i < n; ++i) {
      uint64_t e = (uint64_t)(((u128)i * g) % (2 * n));
      if (e < n) y[e] = x[i];
      else y[e - n] = x[i] ? q - x[i] : 0;
    }
    free(x);
    ntt_limb(q, psi, log_n, y);
  }
}

/* HMUL (Background section): for ciphertexts a = (a0, a1), b = (b0, b1) over
 * the level's Q (NTT form), out = (a0*b0, a0*b1 + a1*b0) + KS(a1*b1), the
 * KeySwitch with the top-level key (from s*s to s).
 * a, b, out [batch][2][level][N]. */
int orc_hmul_level(int dnum, int log_n, int ell, int level, const uint64_t* a, const uint64_t* b,
                   const uint64_t* evk, uint64_t* out, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  size_t n = p.n, L = (size_t)p.ell;
  uint64_t* d2 = (uint64_t*)malloc((size_t)batch * L * n * sizeof(uint64_t));
  uint64_t* ks = (uint64_t*)malloc((size_t)batch * 2 * L * n * sizeof(uint64_t));
  if (!d2 || !ks) { free(d2); free(ks); return -2; }
  for (int bt = 0; bt < batch; ++bt)
    for (size_t i = 0; i < L; ++i) {
      uint64_t q = p.mod[i];
      const uint64_t* a0 = a + ((size_t)bt * 2 * L + i) * n;
      const uint64_t* a1 = a + ((size_t)bt * 2 * L + L + i) * n;
      const uint64_t* b0 = b + ((size_t)bt * 2 * L + i) * n;
      const uint64_t* b1 = b + ((size_t)bt * 2 * L + L + i) * n;
      uint64_t* o0 = out + ((size_t)bt * 2 * L + i) * n;
      uint64_t* o1 = out + ((size_t)bt * 2 * L + L + i) * n;
      for (size_t x = 0; x < n; ++x) {
        o0[x] = mulmod(a0[x], b0[x], q);
        o1[x] = addmod(mulmod(a0[x], b1[x], q), mulmod(a1[x], b0[x], q), q);
        d2[((size_t)bt * L + i) * n + x] = mulmod(a1[x], b1[x], q);
      }
    }
  int rc = orc_keyswitch_level(dnum, log_n, ell, level, d2, evk, ks, batch);
  if (rc == 0)
    for (int bt = 0; bt < batch; ++bt)
      for (size_t c = 0; c < 2; ++c)
        for (size_t i = 0; i < L; ++i) {
          uint64_t q = p.mod[i];
          uint64_t* o = out + (((size_t)bt * 2 + c) * L + i) * n;
          const uint64_t* k = ks + (((size_t)bt * 2 + c) * L + i) * n;
          for (size_t x = 0; x < n; ++x) o[x] = addmod(o[x], k[x], q);
        }
  free(d2);
  free(ks);
  return rc;
}

/* HROT by the automorphism X -> X^g: out = (sigma(c0), 0) + KS(sigma(c1)),
 * the KeySwitch with the top-level key from sigma(s) to s.
 * ct, out [batch][2][level][N].
 * This is a reading of the Background section's formula, which places the
 * rotated second component first and key-switches the rotated first one:
 * with the convention of the HMUL formula next to it (c0 + c1*s, so that
 * the KS term there multiplies s^2), the component to switch is the one
 * that multiplies sigma(s), sigma(c1). */
int orc_hrot_level(int dnum, int log_n, int ell, int level, const uint64_t* ct, uint64_t g, const uint64_t* evk,
                   uint64_t* out, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0 || (g & 1) == 0) return -1;
  size_t n = p.n, L = (size_t)p.ell;
  uint64_t* d = (uint64_t*)malloc((size_t)batch * L * n * sizeof(uint64_t));
  uint64_t* ks = (uint64_t*)malloc((size_t)batch * 2 * L * n * sizeof(uint64_t));
  if (!d || !ks) { free(d); free(ks); return -2; }
  for (int bt = 0; bt < batch; ++bt)
    for (size_t i = 0; i < L; ++i) {
      orc_automorph(p.mod[i], p.psi[i], p.log_n, ct + ((size_t)bt * 2 * L + i) * n, g,
                    out + ((size_t)bt * 2 * L + i) * n, 1);
      orc_automorph(p.mod[i], p.psi[i], p.log_n, ct + ((size_t)bt * 2 * L + L + i) * n, g,
                    d + ((size_t)bt * L + i) * n, 1);
    }
  int rc = orc_keyswitch_level(dnum, log_n, ell, level, d, evk, ks, batch);
  if (rc == 0)
    for (int bt = 0; bt < batch; ++bt)
      for (size_t i = 0; i < L; ++i) {
        uint64_t q = p.mod[i];
        uint64_t* o0 = out + ((size_t)bt * 2 * L + i) * n;
        uint64_t* o1 = out + ((size_t)bt * 2 * L + L + i) * n;
        const uint64_t* k0 = ks + ((size_t)bt * 2 * L + i) * n;
        const uint64_t* k1 = ks + ((size_t)bt * 2 * L + L + i) * n;
        for (size_t x = 0; x < n; ++x) {
          o0[x] = addmod(o0[x], k0[x], q);
          o1[x] = k1[x];
        }
      }
  free(d);
  free(ks);
  return rc;
}

/* Decryption check of a KeySwitch output (test side): per limb q_i,
 * e_i = INTT(out0 + out1*NTT(s2) - d*NTT(s)), read as centered residues.
 * err [batch][N] receives the limb-0 centered values; the return value is 1 if
 * every limb holds the same integer at every coefficient, 0 if not, <0 on error. */
int orc_ks_error_level(int dnum, int log_n, int ell, int level, const uint64_t* d, const uint64_t* out,
                       const int8_t* s, const int8_t* s2, int64_t* err, int batch) {
  orc_params p;
  if (derive_level(dnum, log_n, ell, level, &p) != 0) return -1;
  size_t n = p.n;
  int agree = 1;
  for (int b = 0; b < batch; ++b) {
    const uint64_t* db = d + (size_t)b * p.ell * n;
    const uint64_t* ob = out + (size_t)b * 2 * p.ell * n;
    int64_t* eb = err + (size_t)b * n;
    for (int i = 0; i < p.ell; ++i) {
      uint64_t q = p.mod[i];
      uint64_t* sh = (uint64_t*)malloc(n * sizeof(uint64_t));
      uint64_t* s2h = (uint64_t*)malloc(n * sizeof(uint64_t));
      uint64_t* v = (uint64_t*)malloc(n * sizeof(uint64_t));
      for (size_t x = 0; x < n; ++x) { sh[x] = signed_mod(s[x], q); s2h[x] = signed_mod(s2[x], q); }
      ntt_limb(q, p.psi[i], p.log_n, sh);
      ntt_limb(q, p.psi[i], p.log_n, s2h);
      for (size_t x = 0; x < n; ++x) {
        uint64_t t0 = addmod(ob[(size_t)i * n + x], mulmod(ob[((size_t)p.ell + i) * n + x], s2h[x], q), q);
        v[x] = submod(t0, mulmod(db[(size_t)i * n + x], sh[x], q), q);
      }
      intt_limb(q, p.psi[i], p.log_n, v);
      for (size_t x = 0; x < n; ++x) {
        int64_t c = v[x] > q / 2 ? -(int64_t)(q - v[x]) : (int64_t)v[x];
        if (i == 0) eb[x] = c;
        else if (eb[x] != c) agree = 0;
      }
      free(sh); free(s2h); free(v);
    }
  }
  return agree;
}

int orc_ks_error(int dnum, int log_n, int ell, const uint64_t* d, const uint64_t* out, const int8_t* s,
                 const int8_t* s2, int64_t* err, int batch) {
  return orc_ks_error_level(dnum, log_n, ell, ell, d, out, s, s2, err, batch);
}
