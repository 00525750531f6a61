// Device-side data structures, modular arithmetic and NTT building blocks.
//
// Two arithmetics share the transform code:
//  * ArF, for the Q primes (q < 2^50): residues are held as integer-valued
//    doubles and multiplied with FP64 FMA. For a product p = a*b,
//    h = fl(a*b), l = fma(a, b, -h) gives p = h + l exactly; k = rint(h * fl(1/q))
//    is within 1/2 + 1.5*2^-52*|p|/q of p/q, and r = fma(-k, q, h) + l = p - k*q
//    exactly whenever |p| <= 2^103. So |r| <= q/2 + 1.5*2^-52*|p|. The
//    transform keeps every value within 2q (for q in [2^49, 2^50)), where
//    products of a value and a balanced twiddle (|w| <= q/2) stay below
//    q^2 < 2^100. MI355X runs FP64 FMA at the full vector rate, which makes
//    this about three times faster than 64-bit integer products.
//  * ArI, for the P primes (p < 2^60): uint64 residues; products by fixed
//    constants use Shoup's method (w' = floor(w * 2^64 / q)), products of two
//    variables Montgomery's REDC with R = 2^64. Forward butterflies keep
//    Harvey's [0, 4q) range, inverse butterflies [0, 2q).
// Between kernels, Q-limb data is stored as canonical uint64 residues and
// P-limb data in the lazy integer ranges stated at each kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ks {

// Per-limb constants (one entry per prime of the extended basis).
struct LimbC {
  uint64_t q;
  uint64_t two_q;
  uint64_t mont_ninv;  // -q^-1 mod 2^64
  uint64_t r2;         // 2^128 mod q
  uint64_t ninv, ninv_s;
  uint64_t red_s;      // floor(2^64 / q): Shoup companion of 1
  double qd;           // q as a double (exact for the Q primes)
  double qinv;         // fl(1 / q)
  double ninv_d;       // balanced N^-1 mod q (Q primes)
  uint64_t r64, r64_s; // 2^64 mod q with its Shoup companion
  // Recombination of the int8-MFMA base conversion (see k_modup_cols_mx):
  double r32_d;        // balanced 2^32 mod q (Q primes)
  uint64_t r32, r32_s; // 2^32 mod q with its Shoup companion (P primes)
  uint64_t cadj;       // (-2^51 - 2^83) mod q (P primes)
};

// Every table of one parameter set. Pointers are device addresses after
// upload (offsets into the host blob before it).
struct DevTables {
  int log_n, ell, k, nl, alpha, ndig;
  const LimbC* limb;        // [nl]
  const uint64_t* twf;      // [nl][N][2]: (psi^brv(i), Shoup) for i in [1, N)
  const uint64_t* twi;      // [nl][N][2]: (psi^-brv(i), Shoup)
  const double* twf_d;      // [ell][N]: balanced psi^brv(i) (Q primes)
  const double* twi_d;      // [ell][N]: balanced psi^-brv(i)
  const uint64_t* up_pre;   // [ell][2]: N^-1 * [(D_j/q_i)^-1]_{q_i}, Shoup (j = digit of i)
  const double* up_pre_d;   // [ell]: the same, balanced double
  const uint64_t* up_mat;   // [ell][nl][2]: [D_j/q_i]_t with its Shoup companion mod t
  const double* up_mat_d;   // [ell][ell]: [D_j/q_i]_{q_t}, balanced double (Q targets)
  const uint64_t* dn_pre;   // [k][2]: N^-1 * [(P/p_m)^-1]_{p_m}, Shoup
  const uint64_t* dn_mat;   // [k][ell][2]: [P/p_m]_{q_i}, Shoup mod q_i
  const double* dn_mat_d;   // [k][ell][2]: balanced [2^30 * P/p_m]_{q_i}, [P/p_m]_{q_i}
  const uint64_t* dn_pinv;  // [ell][2]: [P^-1]_{q_i}, Shoup
  const double* dn_pinv_d;  // [ell]: balanced [P^-1]_{q_i}
  const uint64_t* up_hinv;  // [ell][2]: [(D_j/q_i)^-1]_{q_i}, Shoup (no N^-1)
  const uint64_t* dn_hinv;  // [k][2]: [(P/p_m)^-1]_{p_m}, Shoup (no N^-1)
  // Constant operands of the int8-MFMA base conversion: per 4-target group
  // and MFMA step, 16 bytes per lane (see k_modup_cols_mx for the layout).
  const uint64_t* up_mx;    // [ndig][up_ng][up_nm][64][2]
  const uint64_t* dn_mx;    // [dn_ng][dn_nm][64][2]
  int up_ng, up_nm, dn_ng, dn_nm;
  // Rows of the evaluation key [ndig][2][evk_nl][N]: limb t < ell is row t,
  // P limb ell + m is row evk_p0 + m. At the top level evk_nl = nl and
  // evk_p0 = ell; at a lower level the key of the top level is read as is.
  int evk_nl, evk_p0;
};

// Row of limb t of the extended basis in one (digit, component) slice of the key.
__device__ __forceinline__ size_t key_row(const DevTables& tb, int j, int c, int t) {
  return ((size_t)j * 2 + c) * tb.evk_nl + (t < tb.ell ? t : tb.evk_p0 + (t - tb.ell));
}

// ------------------------------------------------------------ integers

__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  // a < 2^64, w < q: returns a*w mod q in [0, 2q).
  const uint64_t hi = __umul64hi(a, ws);
  return a * w - hi * q;
}

__device__ __forceinline__ uint64_t reduce2(uint64_t x, uint64_t q) { return x >= q ? x - q : x; }

__device__ __forceinline__ uint64_t reduce4(uint64_t x, uint64_t q, uint64_t two_q) {
  x = x >= two_q ? x - two_q : x;
  return x >= q ? x - q : x;
}

// Montgomery REDC of a*b for a*b < q * 2^64: returns a*b*2^-64 mod q in [0, 2q).
__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t ninv) {
  const uint64_t lo = a * b, hi = __umul64hi(a, b);
  const uint64_t m = lo * ninv;
  const uint64_t mh = __umul64hi(m, q);
  return hi + mh + (lo != 0 ? 1 : 0);
}

// --------------------------------------------------------------- FP64

// a*b mod q as an integer-valued double with |r| <= q/2 + 1.5*2^-52*|a*b|,
// for |a*b| <= 2^103 (see the header comment).
__device__ __forceinline__ double f_mul(double a, double b, double q, double qinv) {
  const double h = a * b;
  const double l = __fma_rn(a, b, -h);
  const double k = __builtin_rint(h * qinv);
  const double r = __fma_rn(-k, q, h);
  return r + l;
}

// x mod q into [-q/2 - 1, q/2 + 1], for integer-valued |x| < 2^53.
__device__ __forceinline__ double f_red(double x, double q, double qinv) {
  return __fma_rn(-__builtin_rint(x * qinv), q, x);
}

// Exact conversion of an integer 0 <= v < 2^52.
__device__ __forceinline__ double u2d(uint64_t v) {
  return __longlong_as_double((long long)(v | 0x4330000000000000ull)) - 4503599627370496.0;
}

// Canonical residue of an integer-valued |x| < 2^53, as uint64.
__device__ __forceinline__ uint64_t f_canon(double x, double q, double qinv) {
  double r = f_red(x, q, qinv);
  r = r < 0.0 ? r + q : r;
  return (uint64_t)__double_as_longlong(r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// Canonical residue in [0, q) as a double.
__device__ __forceinline__ double f_canon_d(double x, double q, double qinv) {
  const double r = f_red(x, q, qinv);
  return r < 0.0 ? r + q : r;
}

// ------------------------------------------------------ arithmetics

// Read-only table loads through the constant address space: when the
// address is the same for the whole wavefront (column-pass twiddles, BConv
// constants) they become scalar loads into SGPRs, sparing vector registers;
// otherwise they are ordinary vector loads.
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

struct Tw {
  uint64_t w, ws;
};

__device__ __forceinline__ Tw load_tw(const uint64_t* table, uint32_t idx) {
  const ulonglong2 v = reinterpret_cast<const ulonglong2*>(table)[idx];
  return Tw{v.x, v.y};
}

// Integer arithmetic of one P limb; `tw` is its (w, Shoup) table.
struct ArI {
  using T = uint64_t;
  uint64_t q, two_q;
  const uint64_t* tw;
  // Forward (Cooley-Tukey): X, Y in [0, 4q) -> X + W*Y, X - W*Y in [0, 4q).
  __device__ __forceinline__ void fwd(T& X, T& Y, uint32_t idx) const {
    const Tw t = load_tw(tw, idx);
    const uint64_t x = X >= two_q ? X - two_q : X;
    const uint64_t v = mul_shoup(Y, t.w, t.ws, q);
    X = x + v;
    Y = x - v + two_q;
  }
  __device__ __forceinline__ void fwd_lazy(T& X, T& Y, uint32_t idx) const { fwd(X, Y, idx); }
  // Inverse (Gentleman-Sande): X, Y in [0, 2q) -> X + Y, W*(X - Y) in [0, 2q).
  __device__ __forceinline__ void inv(T& X, T& Y, uint32_t idx) const {
    const Tw t = load_tw(tw, idx);
    uint64_t s = X + Y;
    s = s >= two_q ? s - two_q : s;
    const uint64_t d = X - Y + two_q;
    X = s;
    Y = mul_shoup(d, t.w, t.ws, q);
  }
};

// FP64 arithmetic of one Q limb; `tw` is its balanced twiddle table.
// Invariant: every value entering a butterfly satisfies |x| <= 2.2q.
//
// Bounds (q < 2^50, so 1.5 * 2^-52 * |a| * q/2 <= 0.1875 |a| for a product
// with a balanced twiddle): a reducing forward stage maps inputs within B to
// outputs within q + 0.1875 B (+1); a lazy one (X not reduced) to within
// 1.1875 B + 0.5q. The transforms alternate them, starting with a reducing
// stage in every group of stages (sub_fwd), which keeps every value within
// 2.2q: from B <= 2.2q, reduce -> 1.42q, lazy -> 2.18q, reduce -> 1.41q.
// Products stay below 1.1 q^2 < 2^100 and sums below 2^53.
struct ArF {
  using T = double;
  double q, qinv;
  const double* tw;
  // X <- red(X) (|X| <= q/2 + 1); V = W*Y with |V| <= q/2 + 0.1875|Y|.
  __device__ __forceinline__ void fwd(T& X, T& Y, uint32_t idx) const {
    const double w = tw[idx];
    const double x = f_red(X, q, qinv);
    const double v = f_mul(Y, w, q, qinv);
    X = x + v;
    Y = x - v;
  }
  // The same without reducing X (3 instructions fewer).
  __device__ __forceinline__ void fwd_lazy(T& X, T& Y, uint32_t idx) const {
    const double w = tw[idx];
    const double v = f_mul(Y, w, q, qinv);
    const double x = X;
    X = x + v;
    Y = x - v;
  }
  // X + Y reduced (|.| <= q/2 + 1); W*(X - Y) with |X - Y| <= 4q: |.| <= q/2 + 0.75q.
  __device__ __forceinline__ void inv(T& X, T& Y, uint32_t idx) const {
    const double w = tw[idx];
    const double s = X + Y, d = X - Y;
    X = f_red(s, q, qinv);
    Y = f_mul(d, w, q, qinv);
  }
};

// One subproblem of 2^K elements in registers. Local stage rho pairs
// elements at distance 2^(K-1-rho); the twiddle of local group g is entry
// (base << rho) + g of the bit-reversed table, where `base` is the table
// index of the subproblem at its first stage (the butterfly tree of the
// transform numbers node u's children 2u and 2u+1).
// Local stages alternate reducing (even rho) and lazy (odd rho) butterflies.
//
// PS >= 0: the table is a block's staged copy (base = 2^PS + p) whose stages
// PS.. are stored group-major, entry (p << rho) + g of stage PS + rho at
// 2^(PS + rho) + (g << PS) + p, so that the lanes of a wave (consecutive p)
// read consecutive words.
template <int K, int PS = -1, class Ar>
__device__ __forceinline__ void sub_fwd(const Ar& A, typename Ar::T* x, uint32_t base) {
#pragma unroll
  for (int rho = 0; rho < K; ++rho) {
    const int dist = 1 << (K - 1 - rho);
#pragma unroll
    for (int j = 0; j < (1 << K); ++j) {
      if (j & dist) continue;
      const uint32_t g = (uint32_t)(j >> (K - rho));
      const uint32_t idx = PS < 0 ? (base << rho) + g
                                  : base + ((1u << (PS + rho)) - (1u << PS)) + (g << (PS < 0 ? 0 : PS));
      if (rho & 1)
        A.fwd_lazy(x[j], x[j + dist], idx);
      else
        A.fwd(x[j], x[j + dist], idx);
    }
  }
}

template <int K, class Ar>
__device__ __forceinline__ void sub_inv(const Ar& A, typename Ar::T* x, uint32_t base) {
#pragma unroll
  for (int rho = K - 1; rho >= 0; --rho) {
    const int dist = 1 << (K - 1 - rho);
#pragma unroll
    for (int j = 0; j < (1 << K); ++j) {
      if (j & dist) continue;
      A.inv(x[j], x[j + dist], (base << rho) + (uint32_t)(j >> (K - rho)));
    }
  }
}

// Operands of HMUL or HROT folded into a fused KeySwitch (a == nullptr: a
// plain KeySwitch). HMUL: ciphertexts a and b [items][2][ell][N], galois 0.
// HROT: a the ciphertext to rotate, b unused, galois the Galois element.
struct EvalIn {
  const uint64_t* a;
  const uint64_t* b;
  uint32_t galois;
};

// Slot of the input that slot t of sigma_g(x) takes in NTT form (slot t holds
// the evaluation at psi^(2 brv(t) + 1)): 2 brv(t') + 1 = g (2 brv(t) + 1) mod 2N.
__device__ __forceinline__ uint32_t galois_src(uint32_t t, uint32_t g, int log_n) {
  const uint32_t e = 2u * (__brev(t) >> (32 - log_n)) + 1u;
  const uint32_t e2 = (uint32_t)(((uint64_t)g * e) & ((2u << log_n) - 1u));
  return __brev((e2 - 1u) >> 1) >> (32 - log_n);
}

// LDS word of element x: one pad word after every 16, so that the strided
// round layouts hit distinct banks.
__device__ __forceinline__ int lds_pad(int x) { return x + (int)((unsigned)x >> 4); }

// lds_pad(x0 + d) = lds_pad(x0) + d + (d >> 4) for the strides d = j*L of a
// round layout (L a power of two, x0 = pos(r, tid, u, 0)): x0 mod 16 plus
// d mod 16 never reaches 16, since either 16 divides d, or x0 mod 16 < L and
// d mod 16 <= 16 - L, or the whole group of 2^k*L <= 16 elements shares its
// 16-word line. The per-register offsets are then compile-time constants.
__device__ constexpr int pad_step(int d) { return d + (d >> 4); }

// Transform stages log_r .. log_n-1 (forward) of one contiguous block of
// M = 2^LOGM elements, block index b in [0, R). T = M / E threads, E = 2^LOGE
// elements per thread, done in rounds of LOGE stages (the first round takes
// the remainder). Between rounds the block goes through LDS.
//
// Register layouts ("positions"): in round r with first local stage s0 and
// size k, register u*2^k + j of thread tid holds element
//   x = hi * (M >> s0) + lo + j * L,  L = M >> (s0 + k),  p = tid + u*T,
//   lo = p mod L, hi = p / L.
// "FR" is the first round's layout (x = p + j*(M >> K1)); "CL" is the
// coalesced layout x = tid + i*T. Forward transforms take FR and return CL;
// inverse transforms take CL and return FR. Both layouts give consecutive
// threads consecutive addresses for every register, so global loads and
// stores at either end are coalesced; the last round's own layout
// (x = tid*E + j) is transposed through LDS.
template <int LOGM, int LOGE>
struct BlockNtt {
  static constexpr int M = 1 << LOGM;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = M / E;
  static constexpr int NR = (LOGM + LOGE - 1) / LOGE;
  static constexpr int K1 = LOGM - LOGE * (NR - 1);
  static constexpr int LDS_WORDS = M + (M >> 4);
  static_assert(NR >= 2, "a block needs at least two rounds");

  __device__ static constexpr int round_s0(int r) { return r == 0 ? 0 : K1 + (r - 1) * LOGE; }
  __device__ static constexpr int round_k(int r) { return r == 0 ? K1 : LOGE; }

  __device__ static __forceinline__ int pos(int r, int tid, int u, int j) {
    const int s0 = round_s0(r), k = round_k(r);
    const int p = tid + u * T;
    const int L = M >> (s0 + k);
    const int lo = p & (L - 1);
    const int hi = p / L;
    return hi * (M >> s0) + lo + j * L;
  }
  __device__ static __forceinline__ uint32_t base(int r, int tid, int u, uint32_t B0) {
    const int s0 = round_s0(r), k = round_k(r);
    const int p = tid + u * T;
    const int L = M >> (s0 + k);
    return (B0 << s0) + (uint32_t)(p / L);
  }
  __device__ static __forceinline__ int fr_pos(int tid, int i) { return pos(0, tid, i >> K1, i & ((1 << K1) - 1)); }
  __device__ static __forceinline__ int cl_pos(int tid, int i) { return tid + i * T; }

  template <int K, int PS = -1, class Ar>
  __device__ static __forceinline__ void round_fwd(const Ar& A, typename Ar::T* x, int r, int tid, uint32_t B0) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) sub_fwd<K, PS>(A, x + u * (1 << K), base(r, tid, u, B0));
  }
  // First stage of the last round, where every thread has its own twiddles.
  static constexpr int LAST_S0 = LOGM - LOGE;
  template <int K, class Ar>
  __device__ static __forceinline__ void round_inv(const Ar& A, typename Ar::T* x, int r, int tid, uint32_t B0) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) sub_inv<K>(A, x + u * (1 << K), base(r, tid, u, B0));
  }
  __device__ static constexpr int round_l(int r) { return M >> (round_s0(r) + round_k(r)); }
  template <int K, class V>
  __device__ static __forceinline__ void to_lds(const V* x, V* lds, int r, int tid) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) {
      V* b = lds + lds_pad(pos(r, tid, u, 0));
#pragma unroll
      for (int j = 0; j < (1 << K); ++j) b[pad_step(j * round_l(r))] = x[u * (1 << K) + j];
    }
  }
  template <int K, class V>
  __device__ static __forceinline__ void from_lds(V* x, const V* lds, int r, int tid) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) {
      const V* b = lds + lds_pad(pos(r, tid, u, 0));
#pragma unroll
      for (int j = 0; j < (1 << K); ++j) x[u * (1 << K) + j] = b[pad_step(j * round_l(r))];
    }
  }

  // Whether the layout of round q and the next one hold the same elements in
  // each wavefront. In a round whose groups are at most 64 elements apart
  // (L <= 64) with one register subproblem per thread, the 64 threads of wave
  // w hold exactly elements [64E w, 64E (w + 1)), and so in every later
  // round: the exchange between such rounds touches only the wave's own LDS
  // words, and a wave-local ordering point replaces the workgroup barrier.
  __device__ static constexpr bool wave_local(int q) {
    return T <= 64 || ((q >= 1 || K1 == LOGE) && round_l(q) <= 64);
  }
  // Orders the LDS stores before this point against the loads after it: for
  // the whole workgroup, or (local) for this wavefront, whose LDS accesses
  // execute in order.
  __device__ static __forceinline__ void exchange_sync(bool local) {
    if (local) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  // Forward: x enters in FR, leaves in CL. B0 = R + b. Starts with a barrier
  // so the LDS block may be reused right after a previous call. STAGED: the
  // twiddles are a staged copy (B0 = 1) with the last round's stages stored
  // group-major (sub_fwd with PS = LAST_S0).
  template <bool STAGED = false, class Ar>
  __device__ static void fwd(const Ar& A, typename Ar::T* x, typename Ar::T* lds, int tid, uint32_t B0) {
    round_fwd<K1>(A, x, 0, tid, B0);
    __syncthreads();
    to_lds<K1>(x, lds, 0, tid);
#pragma unroll
    for (int r = 1; r < NR; ++r) {
      exchange_sync(wave_local(r - 1));
      from_lds<LOGE>(x, lds, r, tid);
      if (STAGED && r == NR - 1)
        round_fwd<LOGE, LAST_S0>(A, x, r, tid, B0);
      else
        round_fwd<LOGE>(A, x, r, tid, B0);
      to_lds<LOGE>(x, lds, r, tid);
    }
    __syncthreads();
    const typename Ar::T* c = lds + lds_pad(tid);  // CL: x = tid + i*T
#pragma unroll
    for (int i = 0; i < E; ++i) x[i] = c[pad_step(i * T)];
  }

  // Inverse: x enters in CL, leaves in FR.
  template <class Ar>
  __device__ static void inv(const Ar& A, typename Ar::T* x, typename Ar::T* lds, int tid, uint32_t B0) {
    __syncthreads();
    typename Ar::T* c = lds + lds_pad(tid);
#pragma unroll
    for (int i = 0; i < E; ++i) c[pad_step(i * T)] = x[i];
#pragma unroll
    for (int r = NR - 1; r >= 1; --r) {
      exchange_sync(r < NR - 1 && wave_local(r));  // the first read follows the CL stores
      from_lds<LOGE>(x, lds, r, tid);
      round_inv<LOGE>(A, x, r, tid, B0);
      to_lds<LOGE>(x, lds, r, tid);
    }
    exchange_sync(wave_local(0));
    from_lds<K1>(x, lds, 0, tid);
    round_inv<K1>(A, x, 0, tid, B0);
  }
};

}  // namespace ks
