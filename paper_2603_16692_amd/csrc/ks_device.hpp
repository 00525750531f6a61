// Device-side data structures, modular arithmetic and NTT building blocks.
//
// Residues are uint64. Products by fixed constants (twiddles, BConv
// matrices, scale factors) use Shoup's method with a precomputed companion
// w' = floor(w * 2^64 / q); products of two variables (KeyMult) use
// Montgomery's REDC with R = 2^64 followed by a multiplication by
// R^2 mod q. Transforms keep Harvey's lazy ranges: forward butterflies take
// and return values in [0, 4q), inverse butterflies in [0, 2q), which needs
// 4q < 2^64 (every prime here is below 2^60).
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
  uint64_t red_s;      // floor(2^64 / q): Shoup companion of 1, reduces any x < 2^64
  uint64_t pad;
};

// Every table of one parameter set. Pointers are device addresses after
// upload (offsets into the host blob before it).
struct DevTables {
  int log_n, ell, k, nl, alpha, ndig;
  const LimbC* limb;        // [nl]
  const uint64_t* twf;      // [nl][N][2]: (psi^brv(i), Shoup) for i in [1, N)
  const uint64_t* twi;      // [nl][N][2]: (psi^-brv(i), Shoup)
  const uint64_t* up_pre;   // [ell][2]: N^-1 * [(D_j/q_i)^-1]_{q_i}, Shoup (j = digit of i)
  const uint64_t* up_mat;   // [ell][nl][2]: [D_j/q_i]_t with its Shoup companion mod t
  const uint64_t* dn_pre;   // [k][2]: N^-1 * [(P/p_m)^-1]_{p_m}, Shoup
  const uint64_t* dn_mat;   // [k][ell][2]: [P/p_m]_{q_i}, Shoup mod q_i
  const uint64_t* dn_pinv;  // [ell][2]: [P^-1]_{q_i}, Shoup
  const uint64_t* up_hinv;  // [ell][2]: [(D_j/q_i)^-1]_{q_i}, Shoup (no N^-1)
  const uint64_t* dn_hinv;  // [k][2]: [(P/p_m)^-1]_{p_m}, Shoup (no N^-1)
};

__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  // a < 2^64, w < q: returns a*w mod q in [0, 2q).
  uint64_t hi = __umul64hi(a, ws);
  return a * w - hi * q;
}

__device__ __forceinline__ uint64_t reduce2(uint64_t x, uint64_t q) { return x >= q ? x - q : x; }

__device__ __forceinline__ uint64_t reduce4(uint64_t x, uint64_t q, uint64_t two_q) {
  x = x >= two_q ? x - two_q : x;
  return x >= q ? x - q : x;
}

// Montgomery REDC of a*b for a*b < q * 2^64: returns a*b*2^-64 mod q in [0, 2q).
__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t ninv) {
  uint64_t lo = a * b, hi = __umul64hi(a, b);
  uint64_t m = lo * ninv;
  uint64_t mh = __umul64hi(m, q);
  return hi + mh + (lo != 0 ? 1 : 0);
}

struct Tw {
  uint64_t w, ws;
};

__device__ __forceinline__ Tw load_tw(const uint64_t* table, uint32_t idx) {
  const ulonglong2 v = reinterpret_cast<const ulonglong2*>(table)[idx];
  return Tw{v.x, v.y};
}

// Forward (Cooley-Tukey) butterfly: X, Y in [0, 4q) -> X + W*Y, X - W*Y in [0, 4q).
__device__ __forceinline__ void bf_fwd(uint64_t& X, uint64_t& Y, Tw t, uint64_t q, uint64_t two_q) {
  uint64_t x = X >= two_q ? X - two_q : X;
  uint64_t v = mul_shoup(Y, t.w, t.ws, q);
  X = x + v;
  Y = x - v + two_q;
}

// Inverse (Gentleman-Sande) butterfly: X, Y in [0, 2q) -> X + Y, W*(X - Y) in [0, 2q).
__device__ __forceinline__ void bf_inv(uint64_t& X, uint64_t& Y, Tw t, uint64_t q, uint64_t two_q) {
  uint64_t s = X + Y;
  s = s >= two_q ? s - two_q : s;
  uint64_t d = X - Y + two_q;
  X = s;
  Y = mul_shoup(d, t.w, t.ws, q);
}

// One subproblem of 2^K elements in registers. Local stage rho pairs
// elements at distance 2^(K-1-rho); the twiddle of local group g is entry
// (base << rho) + g of the bit-reversed table, where `base` is the table
// index of the subproblem at its first stage (the butterfly tree of the
// transform numbers node u's children 2u and 2u+1).
template <int K>
__device__ __forceinline__ void sub_fwd(uint64_t* x, const uint64_t* tw, uint32_t base, uint64_t q,
                                        uint64_t two_q) {
#pragma unroll
  for (int rho = 0; rho < K; ++rho) {
    const int dist = 1 << (K - 1 - rho);
#pragma unroll
    for (int j = 0; j < (1 << K); ++j) {
      if (j & dist) continue;
      const uint32_t idx = (base << rho) + (uint32_t)(j >> (K - rho));
      bf_fwd(x[j], x[j + dist], load_tw(tw, idx), q, two_q);
    }
  }
}

template <int K>
__device__ __forceinline__ void sub_inv(uint64_t* x, const uint64_t* tw, uint32_t base, uint64_t q,
                                        uint64_t two_q) {
#pragma unroll
  for (int rho = K - 1; rho >= 0; --rho) {
    const int dist = 1 << (K - 1 - rho);
#pragma unroll
    for (int j = 0; j < (1 << K); ++j) {
      if (j & dist) continue;
      const uint32_t idx = (base << rho) + (uint32_t)(j >> (K - rho));
      bf_inv(x[j], x[j + dist], load_tw(tw, idx), q, two_q);
    }
  }
}

__device__ __forceinline__ int lds_pad(int x) { return x + (x >> 4); }

// Transform stages log_r .. log_n-1 (forward) of one contiguous block of
// M = 2^LOGM elements, block index b in [0, R). T = M / E threads, E = 2^LOGE
// elements per thread, done in rounds of LOGE stages (the first round takes
// the remainder). Between rounds the block goes through LDS.
//
// Register layouts ("positions"): in round r with first local stage s0 and
// size k, register u*2^k + j of thread tid holds element
//   x = hi * (M >> s0) + lo + j * L,  L = M >> (s0 + k),  p = tid + u*T,
//   lo = p mod L, hi = p / L.
// The first round's positions ("FR": x = p + j*(M >> K1)) are coalesced for
// global loads and stores; the last round's ("LR": x = tid*E + j) give each
// thread E contiguous elements.
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

  // Element index of register (u, j) in round r.
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
  __device__ static __forceinline__ int fr_pos(int tid, int i) {  // register i in the FR layout
    return pos(0, tid, i >> K1, i & ((1 << K1) - 1));
  }
  __device__ static __forceinline__ int lr_pos(int tid, int i) { return tid * E + i; }

  template <int K>
  __device__ static __forceinline__ void round_fwd(uint64_t* x, int r, int tid, uint32_t B0, const uint64_t* tw,
                                                   uint64_t q, uint64_t two_q) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) sub_fwd<K>(x + u * (1 << K), tw, base(r, tid, u, B0), q, two_q);
  }
  template <int K>
  __device__ static __forceinline__ void round_inv(uint64_t* x, int r, int tid, uint32_t B0, const uint64_t* tw,
                                                   uint64_t q, uint64_t two_q) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u) sub_inv<K>(x + u * (1 << K), tw, base(r, tid, u, B0), q, two_q);
  }
  template <int K>
  __device__ static __forceinline__ void to_lds(const uint64_t* x, uint64_t* lds, int r, int tid) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u)
#pragma unroll
      for (int j = 0; j < (1 << K); ++j) lds[lds_pad(pos(r, tid, u, j))] = x[u * (1 << K) + j];
  }
  template <int K>
  __device__ static __forceinline__ void from_lds(uint64_t* x, const uint64_t* lds, int r, int tid) {
#pragma unroll
    for (int u = 0; u < (E >> K); ++u)
#pragma unroll
      for (int j = 0; j < (1 << K); ++j) x[u * (1 << K) + j] = lds[lds_pad(pos(r, tid, u, j))];
  }

  // Forward: x enters in the FR layout (values in [0, 4q)) and leaves in the
  // LR layout (values in [0, 4q)). B0 = R + b. Starts with a barrier so the
  // LDS block may be reused right after a previous call.
  __device__ static void fwd(uint64_t* x, uint64_t* lds, int tid, uint32_t B0, const uint64_t* tw, uint64_t q,
                             uint64_t two_q) {
    round_fwd<K1>(x, 0, tid, B0, tw, q, two_q);
    __syncthreads();
    to_lds<K1>(x, lds, 0, tid);
#pragma unroll
    for (int r = 1; r < NR; ++r) {
      __syncthreads();
      from_lds<LOGE>(x, lds, r, tid);
      round_fwd<LOGE>(x, r, tid, B0, tw, q, two_q);
      if (r + 1 < NR) to_lds<LOGE>(x, lds, r, tid);
    }
  }

  // Inverse: x enters in the LR layout (values in [0, 2q)) and leaves in the
  // FR layout (values in [0, 2q)).
  __device__ static void inv(uint64_t* x, uint64_t* lds, int tid, uint32_t B0, const uint64_t* tw, uint64_t q,
                             uint64_t two_q) {
    __syncthreads();
#pragma unroll
    for (int r = NR - 1; r >= 1; --r) {
      if (r + 1 < NR) from_lds<LOGE>(x, lds, r, tid);
      round_inv<LOGE>(x, r, tid, B0, tw, q, two_q);
      to_lds<LOGE>(x, lds, r, tid);
      __syncthreads();
    }
    from_lds<K1>(x, lds, 0, tid);
    round_inv<K1>(x, 0, tid, B0, tw, q, two_q);
  }
};

}  // namespace ks
