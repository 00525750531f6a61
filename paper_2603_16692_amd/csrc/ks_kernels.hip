// HIP kernels of the KeySwitch path for gfx950, and their host launchers.
//
// A limb of N = R * M coefficients is transformed in two passes:
//   * a column pass: thread c owns the R coefficients c, c + M, ..., and runs
//     the first log R stages of the forward transform (or the last log R of the
//     inverse) in registers; consecutive threads touch consecutive addresses;
//   * a block pass: a workgroup owns M consecutive coefficients and runs the
//     remaining log M stages through LDS (BlockNtt), with coalesced global
//     loads and stores at both ends.
// ModUp's BConv sits between the inverse column pass and the forward column
// pass of the new limbs (same columns, all in registers), KeyMult follows the
// forward block pass, and ModDown repeats the pattern. Q limbs (q < 2^50) run
// on FP64 arithmetic (ArF), P limbs (p < 2^60) on 64-bit integers (ArI); the
// choice is made per workgroup, since a workgroup works on a single limb.
// Every kernel states the ranges of the values it reads and writes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "ks_device.hpp"
#include "ks_kernels.hpp"

namespace ks {

namespace {

constexpr int TC = 64;  // threads of a column-pass workgroup

__device__ __forceinline__ size_t lane_col() { return (size_t)blockIdx.x * TC + threadIdx.x; }

__device__ __forceinline__ ArF arf(const DevTables& tb, const LimbC& L, int limb, bool inverse) {
  const size_t N = (size_t)1 << tb.log_n;
  return ArF{L.qd, L.qinv, (inverse ? tb.twi_d : tb.twf_d) + (size_t)limb * N};
}
__device__ __forceinline__ ArI ari(const DevTables& tb, const LimbC& L, int limb, bool inverse) {
  const size_t N = (size_t)1 << tb.log_n;
  return ArI{L.q, L.two_q, (inverse ? tb.twi : tb.twf) + (size_t)limb * N * 2};
}

// Canonical double in [0, q) -> uint64.
__device__ __forceinline__ uint64_t d2u(double v) {
  return (uint64_t)__double_as_longlong(v + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// XCD-aware placement of block-pass workgroups. MI355X dispatches workgroup
// w to XCD w mod 8, and each XCD has its own 4 MB L2. A block-pass "tile" is
// one (limb, block) pair; the batch items of a tile read the same twiddles
// and, in KeyMult, the same key blocks. The mapping below puts all items of a
// tile on one XCD at consecutive dispatch slots, so those shared reads are
// served by that XCD's L2 instead of going to HBM once per item.
// Grid: 8 * ceil(ntiles / 8) * items workgroups (1-D).
struct Tile {
  int tile, item;
  bool valid;
};
__device__ __forceinline__ Tile xcd_tile(int ntiles, int items) {
  const int w = blockIdx.x;
  const int xcd = w & 7, local = w >> 3;
  const int item = local % items, unit = local / items;
  const int tile = unit * 8 + xcd;
  return Tile{tile, item, tile < ntiles};
}
inline unsigned xcd_grid(int ntiles, int items) { return (unsigned)(((ntiles + 7) / 8) * 8 * items); }

// BlockNtt::fwd with the thread index hidden from the optimiser: a kernel that
// runs several transforms would otherwise keep every LDS and twiddle address
// of all rounds live from the first transform to the last, which costs more
// registers than recomputing them.
template <class B, bool STAGED = false, class Ar>
__device__ __forceinline__ void fwd_opaque(const Ar& A, typename Ar::T* v, typename Ar::T* ld, int tid,
                                           uint32_t B0) {
  int t = tid;
  asm volatile("" : "+v"(t));
  B::template fwd<STAGED>(A, v, ld, t, B0);
}
template <class B, class Ar>
__device__ __forceinline__ void inv_opaque(const Ar& A, typename Ar::T* v, typename Ar::T* ld, int tid,
                                           uint32_t B0) {
  int t = tid;
  asm volatile("" : "+v"(t));
  B::inv(A, v, ld, t, B0);
}

// ------------------------------------------------------- standalone passes

// Column pass of ks_ntt / ks_intt on x [items][nlimbs][N] (limb r uses prime
// first + r). Q limbs: canonical in and out. P limbs: forward [0, 4q) in and
// out; inverse [0, 2q) in, canonical out. The inverse includes N^-1.
template <int LOGR, bool INV>
__global__ __launch_bounds__(TC) void k_cols(DevTables tb, uint64_t* x, int first, int nlimbs, int log_m) {
  constexpr int R = 1 << LOGR;
  const int M = 1 << log_m;
  const size_t c = lane_col();
  if (c >= (size_t)M) return;
  const int limb = first + blockIdx.y;
  const LimbC L = tb.limb[limb];
  const size_t N = (size_t)M * R;
  uint64_t* a = x + ((size_t)blockIdx.z * nlimbs + blockIdx.y) * N;
  if (limb < tb.ell) {
    const ArF A = arf(tb, L, limb, INV);
    double v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = u2d(a[c + (size_t)i * M]);
    if (!INV) {
      sub_fwd<LOGR>(A, v, 1u);
    } else {
      sub_inv<LOGR>(A, v, 1u);
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = f_mul(v[i], L.ninv_d, L.qd, L.qinv);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) a[c + (size_t)i * M] = f_canon(v[i], L.qd, L.qinv);
  } else {
    const ArI A = ari(tb, L, limb, INV);
    uint64_t v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = a[c + (size_t)i * M];
    if (!INV) {
      sub_fwd<LOGR>(A, v, 1u);
    } else {
      sub_inv<LOGR>(A, v, 1u);
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = reduce2(mul_shoup(v[i], L.ninv, L.ninv_s, L.q), L.q);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) a[c + (size_t)i * M] = v[i];
  }
}

// Block pass of ks_ntt / ks_intt (and of d at the start of ModUp): one block
// of one limb (first + l) of one item per workgroup (placed by xcd_tile),
// src -> dst (may alias).
// Forward: Q canonical in; P [0, 4q) in; canonical out. Inverse: canonical in;
// out Q canonical, P [0, 2q); times N^-1 (canonical) when `scale` is set.
template <int LOGM, int LOGE, bool INV>
__global__ __launch_bounds__((1 << (LOGM - LOGE)), LOGM >= 12 ? 4 : 1) void k_blocks(DevTables tb, const uint64_t* src, uint64_t* dst,
                                                                 int first, int nlimbs, int items, int scale) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * nlimbs, items);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R, lrel = tl.tile / R;
  const int limb = first + lrel;
  const LimbC L = tb.limb[limb];
  const uint32_t B0 = (uint32_t)R + b;
  const size_t off = ((size_t)tl.item * nlimbs + lrel) * N + (size_t)b * B::M;
  const uint64_t* s = src + off;
  uint64_t* d = dst + off;
  if (limb < tb.ell) {
    const ArF A = arf(tb, L, limb, INV);
    double* ld = reinterpret_cast<double*>(lds);
    double v[B::E];
    if (!INV) {
#pragma unroll
      for (int i = 0; i < B::E; ++i) v[i] = u2d(s[B::fr_pos(tid, i)]);
      B::fwd(A, v, ld, tid, B0);
#pragma unroll
      for (int i = 0; i < B::E; ++i) d[B::cl_pos(tid, i)] = f_canon(v[i], L.qd, L.qinv);
    } else {
#pragma unroll
      for (int i = 0; i < B::E; ++i) v[i] = u2d(s[B::cl_pos(tid, i)]);
      B::inv(A, v, ld, tid, B0);
      if (scale) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = f_mul(v[i], L.ninv_d, L.qd, L.qinv);
      }
#pragma unroll
      for (int i = 0; i < B::E; ++i) d[B::fr_pos(tid, i)] = f_canon(v[i], L.qd, L.qinv);
    }
  } else {
    const ArI A = ari(tb, L, limb, INV);
    uint64_t v[B::E];
    if (!INV) {
#pragma unroll
      for (int i = 0; i < B::E; ++i) v[i] = s[B::fr_pos(tid, i)];
      B::fwd(A, v, lds, tid, B0);
#pragma unroll
      for (int i = 0; i < B::E; ++i) d[B::cl_pos(tid, i)] = reduce4(v[i], L.q, L.two_q);
    } else {
#pragma unroll
      for (int i = 0; i < B::E; ++i) v[i] = s[B::cl_pos(tid, i)];
      B::inv(A, v, lds, tid, B0);
      if (scale) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = reduce2(mul_shoup(v[i], L.ninv, L.ninv_s, L.q), L.q);
      }
#pragma unroll
      for (int i = 0; i < B::E; ++i) d[B::fr_pos(tid, i)] = v[i];
    }
  }
}

// The first pass of a fused HMUL or HROT (in place of the inverse block pass
// of d): one block of one Q limb of one item per workgroup computes d = a1 b1
// (HMUL) or d = sigma_g(c1) (HROT, a gather in NTT form), stores it (the
// digit-parallel last pass reads it as its own digit) and runs the inverse
// block pass into t1, as k_blocks<INV> does for d.
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE)), LOGM >= 12 ? 4 : 1) void k_eval_blocks(
    DevTables tb, EvalIn ev, uint64_t* d2, uint64_t* t1, int items) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM), ell = tb.ell;
  const Tile tl = xcd_tile(R * ell, items);
  if (!tl.valid) return;
  const int tid = threadIdx.x, blk = tl.tile % R, i = tl.tile / R;
  const LimbC L = tb.limb[i];
  const size_t boff = (size_t)blk * B::M;
  const uint64_t* a1 = ev.a + (((size_t)tl.item * 2 + 1) * ell + i) * N;  // the limb's component 1
  const size_t off = ((size_t)tl.item * ell + i) * N + boff;
  double v[B::E];
  if (ev.galois) {
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      const int x = B::cl_pos(tid, e);
      const uint64_t c = a1[galois_src((uint32_t)(boff + x), ev.galois, tb.log_n)];
      d2[off + x] = c;
      v[e] = u2d(c);
    }
  } else {
    const uint64_t* b1 = ev.b + (((size_t)tl.item * 2 + 1) * ell + i) * N;
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      const int x = B::cl_pos(tid, e);
      const uint64_t c = f_canon(f_mul(u2d(a1[boff + x]), u2d(b1[boff + x]), L.qd, L.qinv), L.qd, L.qinv);
      d2[off + x] = c;
      v[e] = u2d(c);
    }
  }
  B::inv(arf(tb, L, i, true), v, reinterpret_cast<double*>(lds), tid, (uint32_t)(R + blk));
#pragma unroll
  for (int e = 0; e < B::E; ++e) t1[off + B::fr_pos(tid, e)] = f_canon(v[e], L.qd, L.qinv);
}

// The HMUL or HROT part of one output element pair of limb i, added to a
// ModDown output (o0, o1) before its final reduction: (a0 b0, a0 b1 + a1 b0)
// or (sigma_g(c0), 0). r0 / r1 index component 0 / 1 of the item's limb i,
// slot t the element's slot in the limb.
template <bool HROT>
__device__ __forceinline__ void add_eval(const LimbC& L, const EvalIn& ev, size_t r0, size_t r1, uint32_t t,
                                         int log_n, double& o0, double& o1) {
  if constexpr (HROT) {
    o0 += u2d(ev.a[r0 - t + galois_src(t, ev.galois, log_n)]);
    return;
  }
  const double a0 = u2d(ev.a[r0]), a1 = u2d(ev.a[r1]), b0 = u2d(ev.b[r0]), b1 = u2d(ev.b[r1]);
  o0 += f_mul(a0, b0, L.qd, L.qinv);
  o1 += f_mul(a0, b1, L.qd, L.qinv) + f_mul(a1, b0, L.qd, L.qinv);
}

// ------------------------------------------------------------ ModUp (K2)

// A column-pass workgroup: 8 waves over the same 64 columns (the 64 lanes).
// Sources are converted once into LDS (wave w takes sources w, w+8, ...);
// after a barrier the waves split the target limbs the same way, so the
// registers a thread needs do not grow with the number of sources.
constexpr int CW = 8;               // waves per column workgroup
constexpr int CT = CW * TC;         // threads per column workgroup

// Digit j = j0 + blockIdx.y of item blockIdx.z, columns blockIdx.x*64 + lane:
// inverse column pass of the digit's limbs of t1 (the block-pass output of d,
// canonical), times N^-1 [(D_j/q_i)^-1]_{q_i}, giving canonical y_i (in LDS,
// [alpha][R][64] doubles); then for every target limb t in [tgt0, tgt1)
// outside D_j: z_t = sum_i y_i [D_j/q_i]_t, forward column pass, store into
// ext1 [items][nslots][nl][N] at slot (slot_stride ? j : 0). Q targets are
// stored canonical, P targets in [0, 4q).
template <int LOGR>
__global__ __launch_bounds__(CT, LOGR <= 4 ? 4 : 2) void k_modup_cols(DevTables tb, const uint64_t* t1, uint64_t* ext1, int j0,
                                                   int nslots, int slot_stride, int tgt0, int tgt1, int log_m) {
  constexpr int R = 1 << LOGR;
  extern __shared__ double ys[];
  const int M = 1 << log_m;
  const size_t N = (size_t)M * R;
  const int lane = threadIdx.x & (TC - 1), wv = threadIdx.x / TC;
  const size_t c = (size_t)blockIdx.x * TC + lane;
  const bool live = c < (size_t)M;
  const int j = j0 + blockIdx.y;
  const int item = blockIdx.z;
  const int ell = tb.ell, nl = tb.nl;
  const int lo = j * tb.alpha;
  const int na = min(lo + tb.alpha, ell) - lo;
  if (live) {
    for (int s = wv; s < na; s += CW) {
      const int i = lo + s;
      const LimbC L = tb.limb[i];
      const uint64_t* a = t1 + ((size_t)item * ell + i) * N;
      double v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = u2d(a[c + (size_t)r * M]);
      sub_inv<LOGR>(arf(tb, L, i, true), v, 1u);
      const double w = tb.up_pre_d[i];
#pragma unroll
      for (int r = 0; r < R; ++r) ys[(s * R + r) * TC + lane] = f_canon_d(f_mul(v[r], w, L.qd, L.qinv), L.qd, L.qinv);
    }
  }
  __syncthreads();
  if (!live) return;
  const int slot = slot_stride ? j : 0;
  uint64_t* e = ext1 + ((size_t)item * nslots + slot) * (size_t)nl * N;
  int u = 0;  // index of the target among those outside D_j
  for (int t = tgt0; t < tgt1; ++t) {
    if (t >= lo && t < lo + na) continue;
    if ((u++ % CW) != wv) continue;
    const LimbC L = tb.limb[t];
    uint64_t* o = e + (size_t)t * N;
    if (t < ell) {
      // |y * c| <= 2^50 * 2^49: each product is within 0.875q; fold every 8
      double z[R];
#pragma unroll
      for (int r = 0; r < R; ++r) z[r] = 0.0;
      for (int s = 0; s < na; ++s) {
        const double cst = ldc(tb.up_mat_d + (size_t)(lo + s) * ell + t);
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] += f_mul(ys[(s * R + r) * TC + lane], cst, L.qd, L.qinv);
        if ((s & 7) == 7) {
#pragma unroll
          for (int r = 0; r < R; ++r) z[r] = f_red(z[r], L.qd, L.qinv);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) z[r] = f_red(z[r], L.qd, L.qinv);
      sub_fwd<LOGR>(arf(tb, L, t, false), z, 1u);
#pragma unroll
      for (int r = 0; r < R; ++r) o[c + (size_t)r * M] = f_canon(z[r], L.qd, L.qinv);
    } else {
      uint64_t z[R];
#pragma unroll
      for (int r = 0; r < R; ++r) z[r] = 0;
      for (int s = 0; s < na; ++s) {
        const size_t ci = 2 * ((size_t)(lo + s) * nl + t);
        const uint64_t w = ldc(tb.up_mat + ci), ws = ldc(tb.up_mat + ci + 1);
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] += reduce2(mul_shoup(d2u(ys[(s * R + r) * TC + lane]), w, ws, L.q), L.q);
        if ((s & 7) == 7) {  // keep the sum below 8q < 2^63
#pragma unroll
          for (int r = 0; r < R; ++r) z[r] = reduce2(mul_shoup(z[r], 1, L.red_s, L.q), L.q);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) z[r] = reduce2(mul_shoup(z[r], 1, L.red_s, L.q), L.q);
      sub_fwd<LOGR>(ari(tb, L, t, false), z, 1u);
#pragma unroll
      for (int r = 0; r < R; ++r) o[c + (size_t)r * M] = z[r];
    }
  }
}

// ------------------------------------------- int8-MFMA base conversion

// BConv as an exact integer contraction on the matrix cores. Each residue
// y < 2^60 is written in balanced base-256 digits y = sum_a d_a 256^a
// (d_a in [-128, 127], signed bytes), and each constant c_{s,t} is folded
// with the digit weight, c'_{s,a,t} = [c_{s,t} 256^a]_t, and split the same
// way into bytes e_{s,a,t,b}. Then
//   sum_s y_s c_{s,t} = sum_b 256^b C_b  (mod t),  C_b = sum_{s,a} d_{s,a} e_{s,a,t,b},
// and every C_b is one entry of an int8 x int8 -> int32 matrix product with
// K = 8 * (number of sources): rows (t, b) come from the constant table,
// columns are coefficients. |C_b| <= 8 * 16 * 128 * 128 = 2^21 for up to 16
// sources. A 32-row tile covers four targets; the host's row order puts all
// eight C_b of targets 2h and 2h+1 in the accumulators of lane half h
// (accumulator i = byte i % 8 of target 2h + i / 8).
// MFMA v_mfma_i32_32x32x32_i8: lane l supplies 16 bytes of row (or column)
// l % 32 at K offsets 16 * (l / 32) .. +15, i.e. sources 4m + 2(l/32) + {0, 1}
// of step m, eight digit bytes each.
typedef int mx_v4i __attribute__((ext_vector_type(4)));
typedef int mx_v16i __attribute__((ext_vector_type(16)));

// Signed bytes of the balanced digits of v < 2^60 (byte 7 is below 18):
// adding 128 to each of the seven low bytes makes them the unsigned bytes of
// v + 0x0080...80; flipping their top bit subtracts the 128 again modulo 256.
__device__ __forceinline__ uint64_t mx_pack(uint64_t v) {
  return (v + 0x0080808080808080ull) ^ 0x0080808080808080ull;
}

__device__ __forceinline__ mx_v16i mx_step(const ulonglong2& a, const ulonglong2& b, const mx_v16i& acc) {
  const mx_v4i av = {(int)(uint32_t)a.x, (int)(uint32_t)(a.x >> 32), (int)(uint32_t)a.y, (int)(uint32_t)(a.y >> 32)};
  const mx_v4i bv = {(int)(uint32_t)b.x, (int)(uint32_t)(b.x >> 32), (int)(uint32_t)b.y, (int)(uint32_t)(b.y >> 32)};
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc, 0, 0, 0);
}

// The target whose partial sums start at accumulator BASE (0 or 8), as
// lo = C0 + 2^8 C1 + 2^16 C2 + 2^24 C3 and hi = C4 + ... + 2^24 C7, exact
// doubles below 2^46.1 in magnitude (the sum is lo + 2^32 hi).
template <int BASE>
__device__ __forceinline__ void mx_halves(const mx_v16i& acc, double& lo, double& hi) {
  const int a0 = acc[BASE + 0] + acc[BASE + 1] * 256, a1 = acc[BASE + 2] + acc[BASE + 3] * 256;
  const int b0 = acc[BASE + 4] + acc[BASE + 5] * 256, b1 = acc[BASE + 6] + acc[BASE + 7] * 256;
  lo = __fma_rn((double)a1, 65536.0, (double)a0);
  hi = __fma_rn((double)b1, 65536.0, (double)b0);
}

// lo + 2^32 hi mod q for a Q prime: |result| <= q/2 + 1.
__device__ __forceinline__ double mx_fold_q(double lo, double hi, double q, double qinv, double r32) {
  return f_red(lo + f_mul(hi, r32, q, qinv), q, qinv);
}

// lo + 2^32 hi mod p for a P prime, in [0, 4p): with u = x + 2^51 >= 0 read
// from the mantissa of x + 1.5 * 2^52, the value is
// u_lo + 2^32 u_hi - 2^51 - 2^83, and cadj = (-2^51 - 2^83) mod p.
__device__ __forceinline__ uint64_t mx_fold_p(double lo, double hi, const LimbC& L) {
  const uint64_t ul = (uint64_t)__double_as_longlong(lo + 6755399441055744.0) & 0x000FFFFFFFFFFFFFull;
  const uint64_t uh = (uint64_t)__double_as_longlong(hi + 6755399441055744.0) & 0x000FFFFFFFFFFFFFull;
  return ul + mul_shoup(uh, L.r32, L.r32_s, L.q) + L.cadj;
}

// Phase 2 of the MFMA column kernels for one target group. A lane in half h
// holds the partial sums of targets 2h and 2h + 1 of the group; each is
// finished in its own pass (PASS 0: accumulators 0..7, PASS 1: 8..15), which
// runs the nm MFMA steps of every row r over the packed digits yp
// ([pairs][R][64] x 16 bytes) again, so that only one target's R values are
// live: for each row the fold mod t, then the forward column pass and, if
// `st`, the store of the R rows. Q groups store canonical residues, P groups
// values in [0, 4p). The raised digits (and ModDown's t2) outgrow the caches,
// so the stores are non-temporal (measured: 5% off the ModUp column kernel).
template <int LOGR, bool QG, int NM, int PASS>
__device__ __forceinline__ void mx_target(const DevTables& tb, const ulonglong2* yp, const ulonglong2 (&cst)[NM],
                                          int t0, int t1, bool st, uint64_t* o, size_t cc, int M) {
  constexpr int R = 1 << LOGR;
  const int lane = threadIdx.x & (TC - 1), h = lane >> 5;
  const int ycol = ((threadIdx.x / TC) & 1) * 32 + (lane & 31);
  const int t = h ? t1 : t0;
  const LimbC& L = tb.limb[t];
  const size_t N = (size_t)M * R;
  using T = typename std::conditional<QG, double, uint64_t>::type;
  T z[R];
  const double q = L.qd, qi = L.qinv, r32 = L.r32_d;
  int yo = h * R * TC + ycol;  // digit words of row r of step m: yp[yo + 2 m R TC + r TC]
#pragma unroll
  for (int r = 0; r < R; ++r) {
    mx_v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < NM; ++m) acc = mx_step(cst[m], yp[yo + (2 * m * R + r) * TC], acc);
    double lo, hi;
    mx_halves<8 * PASS>(acc, lo, hi);
    if constexpr (QG)
      z[r] = mx_fold_q(lo, hi, q, qi, r32);
    else
      z[r] = mx_fold_p(lo, hi, L);
    // One row at a time: this row's result is materialised here (the compiler
    // would otherwise sink the folds below the loop and keep every row's
    // accumulators live), and the next row's digit loads wait for it.
    asm volatile("" : "+v"(z[r]), "+v"(yo));
  }
  if constexpr (QG) {
    sub_fwd<LOGR>(ArF{q, qi, tb.twf_d + (size_t)t * N}, z, 1u);
    if (st) {
#pragma unroll
      for (int r = 0; r < R; ++r) __builtin_nontemporal_store(f_canon(z[r], q, qi), o + cc + (size_t)r * M);
    }
  } else {
    sub_fwd<LOGR>(ArI{L.q, L.two_q, tb.twf + (size_t)t * N * 2}, z, 1u);
    if (st) {
#pragma unroll
      for (int r = 0; r < R; ++r) __builtin_nontemporal_store(z[r], o + cc + (size_t)r * M);
    }
  }
}

// lt[4]: the group's four limbs (padding slots replaced by a stand-in limb,
// wave-uniform); lane half h finishes targets lt[2h] (stored if sa, at oa)
// and lt[2h + 1] (if sb, at ob).
template <int LOGR, bool QG, int NM>
__device__ __forceinline__ void mx_group(const DevTables& tb, const ulonglong2* yp, const ulonglong2* cst_g,
                                         const int (&lt)[4], bool sa, bool sb, uint64_t* oa, uint64_t* ob,
                                         size_t cc, int M) {
  const int lane = threadIdx.x & (TC - 1);
  ulonglong2 cst[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) cst[m] = cst_g[m * 64 + lane];
  mx_target<LOGR, QG, NM, 0>(tb, yp, cst, lt[0], lt[2], sa, oa, cc, M);
  mx_target<LOGR, QG, NM, 1>(tb, yp, cst, lt[1], lt[3], sb, ob, cc, M);
}

// ModUp columns with the int8-MFMA BConv: same arguments and output as
// k_modup_cols. Phase 1 (wave w: sources w, w + 8, ... < 4 nm): inverse
// column pass and pre-scale as in k_modup_cols, canonical y packed into LDS
// as [pair][R][64] x 16 bytes (pair p = sources 2p, 2p + 1; zero past the
// digit's sources and for columns past M). Phase 2: wave w takes the column
// half w % 2 (lane l works on column (w % 2) * 32 + l % 32 of the workgroup)
// and the target groups w/2, w/2 + 4, ...: per digit the Q targets outside
// D_j in groups of four (in basis order), then the P targets.
template <int LOGR, int NM>
__global__ __launch_bounds__(CT, LOGR == 4 ? 4 : 1) void k_modup_cols_mx(DevTables tb, const uint64_t* t1, uint64_t* ext1, int j0,
                                                     int nslots, int slot_stride, int tgt0, int tgt1, int log_m) {
  constexpr int R = 1 << LOGR;
  extern __shared__ ulonglong2 yp[];
  const int M = 1 << log_m;
  const size_t N = (size_t)M * R;
  const int lane = threadIdx.x & (TC - 1), wv = threadIdx.x / TC;
  const size_t c = (size_t)blockIdx.x * TC + lane;
  const bool live = c < (size_t)M;
  const int j = j0 + blockIdx.y;
  const int item = blockIdx.z;
  const int ell = tb.ell, nl = tb.nl, k = tb.k;
  const int lo = j * tb.alpha;
  const int na = min(lo + tb.alpha, ell) - lo;
  constexpr int nm = NM;  // = tb.up_nm
  uint64_t* yw = reinterpret_cast<uint64_t*>(yp);
  for (int s = wv; s < 4 * nm; s += CW) {
    uint64_t y[R];
    if (live && s < na) {
      const int i = lo + s;
      const LimbC L = tb.limb[i];
      const uint64_t* a = t1 + ((size_t)item * ell + i) * N;
      double v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = u2d(a[c + (size_t)r * M]);
      sub_inv<LOGR>(arf(tb, L, i, true), v, 1u);
      const double w = tb.up_pre_d[i];
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = mx_pack(d2u(f_canon_d(f_mul(v[r], w, L.qd, L.qinv), L.qd, L.qinv)));
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) yw[((size_t)((s >> 1) * R + r) * TC + lane) * 2 + (s & 1)] = y[r];
  }
  __syncthreads();
  const int h = lane >> 5;
  const size_t cc = (size_t)blockIdx.x * TC + (wv & 1) * 32 + (lane & 31);
  const bool clive = cc < (size_t)M;
  const int slot = slot_stride ? j : 0;
  uint64_t* e = ext1 + ((size_t)item * nslots + slot) * (size_t)nl * N;
  const int nq = ell - na, nqg = (nq + 3) >> 2, ng = nqg + ((k + 3) >> 2);
  const ulonglong2* cst_j = reinterpret_cast<const ulonglong2*>(tb.up_mx) + (size_t)j * tb.up_ng * nm * 64;
  for (int g = wv >> 1; g < ng; g += CW / 2) {
    const bool qg = g < nqg;
    int tg[4];
    bool any = false;
#pragma unroll
    for (int tau = 0; tau < 4; ++tau) {
      int t = -1;
      if (qg) {
        const int u = 4 * g + tau;
        if (u < nq) t = u < lo ? u : u + na;
      } else {
        const int v = 4 * (g - nqg) + tau;
        if (v < k) t = ell + v;
      }
      tg[tau] = t;
      any = any || (t >= tgt0 && t < tgt1);
    }
    if (!any) continue;
    const int ta = tg[2 * h], tb2 = tg[2 * h + 1];
    const bool sa = clive && ta >= tgt0 && ta < tgt1;
    const bool sb = clive && tb2 >= tgt0 && tb2 < tgt1;
    const int pad = qg ? 0 : ell;  // stand-in limb for padding slots (never stored)
    int lt[4];
#pragma unroll
    for (int tau = 0; tau < 4; ++tau) lt[tau] = tg[tau] >= 0 ? tg[tau] : pad;
    uint64_t* oa = e + (size_t)lt[2 * h] * N;
    uint64_t* ob = e + (size_t)lt[2 * h + 1] * N;
    if (qg)
      mx_group<LOGR, true, NM>(tb, yp, cst_j + (size_t)g * nm * 64, lt, sa, sb, oa, ob, cc, M);
    else
      mx_group<LOGR, false, NM>(tb, yp, cst_j + (size_t)g * nm * 64, lt, sa, sb, oa, ob, cc, M);
  }
}

// ---------------------------------------------------------- KeyMult (K3)

// One block b of one target limb t in [tgt0, tgt0 + ntgt) of one item per
// workgroup (placed by xcd_tile): for every
// digit j in [j0, j1): ext_j = (t in D_j) ? d : forward block pass of ext1;
// s_c += ext_j * evk[j][c]. Then v_c = s_c (+ the previous acc if
// `accumulate`), stored canonical. With `finalize` and t a P limb, the inverse
// block pass of ModDown runs on v_c and leaves [0, 2q) in acc.
// QPATH selects the Q-limb (FP64) or the P-limb (integer) body; the two are
// separate kernels so that each gets its own register allocation.
// With 8 elements per thread at M >= 2^12 the kernel fits 128 registers,
// which lets four waves share each SIMD.
template <int LOGM, int LOGE, bool QPATH>
__global__ __launch_bounds__((1 << (LOGM - LOGE)), (LOGE == 3 && LOGM >= 12) ? 4 : 1) void k_keymult_blocks(
    DevTables tb, const uint64_t* d, const uint64_t* ext1, const uint64_t* evk, uint64_t* acc, int j0, int j1,
    int nslots, int slot_stride, int tgt0, int ntgt, int items, int accumulate, int finalize) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * ntgt, items);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R;
  const int t = tgt0 + tl.tile / R;
  const int item = tl.item;
  const LimbC L = tb.limb[t];
  const uint32_t B0 = (uint32_t)R + b;
  const int nl = tb.nl;
  const size_t boff = (size_t)b * B::M;
  uint64_t* a0 = acc + (((size_t)item * 2 + 0) * nl + t) * N + boff;
  uint64_t* a1 = acc + (((size_t)item * 2 + 1) * nl + t) * N + boff;
  if constexpr (QPATH) {
    const ArF A = arf(tb, L, t, false);
    double* ld = reinterpret_cast<double*>(lds);
    double s0[B::E], s1[B::E], v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) s0[i] = s1[i] = 0.0;
    for (int j = j0; j < j1; ++j) {
      const int lo = j * tb.alpha;
      if (t >= lo && t < lo + tb.alpha) {
        const uint64_t* src = d + ((size_t)item * tb.ell + t) * N + boff;
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = u2d(src[B::cl_pos(tid, i)]);
      } else {
        const int slot = slot_stride ? j : 0;
        const uint64_t* src = ext1 + (((size_t)item * nslots + slot) * nl + t) * N + boff;
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = u2d(src[B::fr_pos(tid, i)]);
        fwd_opaque<B>(A, v, ld, tid, B0);
      }
      const uint64_t* k0 = evk + key_row(tb, j, 0, t) * N + boff;
      const uint64_t* k1 = evk + key_row(tb, j, 1, t) * N + boff;
      // |v| <= 2.2q, key < q: each product is within 1.33q; fold every 4 digits
#pragma unroll
      for (int i = 0; i < B::E; ++i) {
        const int x = B::cl_pos(tid, i);
        s0[i] += f_mul(v[i], u2d(k0[x]), L.qd, L.qinv);
        s1[i] += f_mul(v[i], u2d(k1[x]), L.qd, L.qinv);
      }
      if (((j - j0) & 3) == 3) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
          s0[i] = f_red(s0[i], L.qd, L.qinv);
          s1[i] = f_red(s1[i], L.qd, L.qinv);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
      const int x = B::cl_pos(tid, i);
      double u0 = f_red(s0[i], L.qd, L.qinv), u1 = f_red(s1[i], L.qd, L.qinv);
      if (accumulate) {
        u0 += u2d(a0[x]);
        u1 += u2d(a1[x]);
      }
      a0[x] = f_canon(u0, L.qd, L.qinv);
      a1[x] = f_canon(u1, L.qd, L.qinv);
    }
  } else {
  const ArI A = ari(tb, L, t, false);
  uint64_t s0[B::E], s1[B::E], v[B::E];
#pragma unroll
  for (int i = 0; i < B::E; ++i) s0[i] = s1[i] = 0;
  for (int j = j0; j < j1; ++j) {
    const int slot = slot_stride ? j : 0;
    const uint64_t* src = ext1 + (((size_t)item * nslots + slot) * nl + t) * N + boff;
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = src[B::fr_pos(tid, i)];
    fwd_opaque<B>(A, v, lds, tid, B0);
    const uint64_t* k0 = evk + key_row(tb, j, 0, t) * N + boff;
    const uint64_t* k1 = evk + key_row(tb, j, 1, t) * N + boff;
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
      const int x = B::cl_pos(tid, i);
      // running sums stay in [0, 2q): each Montgomery product is in [0, 2q)
      s0[i] += mont_mul(v[i], k0[x], L.q, L.mont_ninv);
      s0[i] = s0[i] >= L.two_q ? s0[i] - L.two_q : s0[i];
      s1[i] += mont_mul(v[i], k1[x], L.q, L.mont_ninv);
      s1[i] = s1[i] >= L.two_q ? s1[i] - L.two_q : s1[i];
    }
  }
#pragma unroll
  for (int i = 0; i < B::E; ++i) {
    // s < 2q, so s * r2 < 2 q^2 < q * 2^64
    s0[i] = reduce2(mont_mul(s0[i], L.r2, L.q, L.mont_ninv), L.q);
    s1[i] = reduce2(mont_mul(s1[i], L.r2, L.q, L.mont_ninv), L.q);
  }
  if (accumulate) {
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
      const int x = B::cl_pos(tid, i);
      s0[i] = reduce2(s0[i] + a0[x], L.q);
      s1[i] = reduce2(s1[i] + a1[x], L.q);
    }
  }
  if (finalize) {
    const ArI Ai = ari(tb, L, t, true);
    inv_opaque<B>(Ai, s0, lds, tid, B0);
#pragma unroll
    for (int i = 0; i < B::E; ++i) a0[B::fr_pos(tid, i)] = s0[i];
    inv_opaque<B>(Ai, s1, lds, tid, B0);
#pragma unroll
    for (int i = 0; i < B::E; ++i) a1[B::fr_pos(tid, i)] = s1[i];
  } else {
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
      const int x = B::cl_pos(tid, i);
      a0[x] = s0[i];
      a1[x] = s1[i];
    }
  }
  }
}

// ---------------------------------------------------------- ModDown (K4)

// Component blockIdx.y of item blockIdx.z, columns blockIdx.x*64 + lane:
// inverse column pass of the k P limbs (accp [items][2][nl][N] at limbs ell..,
// values in [0, 2q)), times N^-1 [(P/p_m)^-1]: canonical y_m < 2^60 in LDS
// ([k][R][64] uint64). Then for Q limbs i in [tgt0, tgt1), split over the
// waves: z_i = sum_m y_m [P/p_m]_{q_i}, computed in FP64 as
// y_hi [2^30 P/p_m] + y_lo [P/p_m] with y_m = y_hi 2^30 + y_lo; forward column
// pass; t2 [items][2][ell][N] canonical.
template <int LOGR>
__global__ __launch_bounds__(CT, LOGR <= 4 ? 4 : 2) void k_moddown_cols(DevTables tb, const uint64_t* accp, uint64_t* t2, int tgt0,
                                                     int tgt1, int log_m) {
  constexpr int R = 1 << LOGR;
  extern __shared__ uint64_t yl[];
  const int M = 1 << log_m;
  const size_t N = (size_t)M * R;
  const int lane = threadIdx.x & (TC - 1), wv = threadIdx.x / TC;
  const size_t c = (size_t)blockIdx.x * TC + lane;
  const bool live = c < (size_t)M;
  const int comp = blockIdx.y, item = blockIdx.z;
  const int ell = tb.ell, nl = tb.nl, k = tb.k;
  if (live) {
    for (int m = wv; m < k; m += CW) {
      const LimbC L = tb.limb[ell + m];
      const uint64_t* a = accp + (((size_t)item * 2 + comp) * nl + ell + m) * N;
      uint64_t v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = a[c + (size_t)r * M];
      sub_inv<LOGR>(ari(tb, L, ell + m, true), v, 1u);
      const uint64_t w = tb.dn_pre[2 * m], ws = tb.dn_pre[2 * m + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) yl[(m * R + r) * TC + lane] = reduce2(mul_shoup(v[r], w, ws, L.q), L.q);
    }
  }
  __syncthreads();
  if (!live) return;
  for (int i = tgt0 + wv; i < tgt1; i += CW) {
    const LimbC L = tb.limb[i];
    double z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = 0.0;
    for (int m = 0; m < k; ++m) {
      const double ch = tb.dn_mat_d[2 * ((size_t)m * ell + i)];
      const double cl = tb.dn_mat_d[2 * ((size_t)m * ell + i) + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // |y_hi * c|, |y_lo * c| <= 2^79: each product is within q/2 + 1
        const uint64_t yv = yl[(m * R + r) * TC + lane];
        const double yh = (double)(uint32_t)(yv >> 30);
        const double ylo = (double)(uint32_t)(yv & 0x3FFFFFFFull);
        z[r] += f_mul(yh, ch, L.qd, L.qinv) + f_mul(ylo, cl, L.qd, L.qinv);
      }
      if ((m & 3) == 3) {
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] = f_red(z[r], L.qd, L.qinv);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = f_red(z[r], L.qd, L.qinv);
    sub_fwd<LOGR>(arf(tb, L, i, false), z, 1u);
    uint64_t* o = t2 + (((size_t)item * 2 + comp) * ell + i) * N;
#pragma unroll
    for (int r = 0; r < R; ++r) o[c + (size_t)r * M] = f_canon(z[r], L.qd, L.qinv);
  }
}

// ModDown columns with the int8-MFMA BConv: same arguments and output as
// k_moddown_cols. Phase 1 (wave w: P limbs w, w + 8, ... < 4 nm): inverse
// column pass of acc_P and the scale by N^-1 [(P/p_m)^-1]_{p_m} as in
// k_moddown_cols, canonical y packed into LDS ([pair][R][64] x 16 bytes,
// zero past the k sources and for columns past M). Phase 2: wave w takes the
// column half w % 2 and the groups of four Q limbs w/2, w/2 + 4, ... that
// meet [tgt0, tgt1); output t2 canonical.
template <int LOGR, int NM>
__global__ __launch_bounds__(CT, LOGR == 4 ? 4 : 1) void k_moddown_cols_mx(DevTables tb, const uint64_t* accp, uint64_t* t2, int tgt0,
                                                       int tgt1, int log_m) {
  constexpr int R = 1 << LOGR;
  extern __shared__ ulonglong2 yp[];
  const int M = 1 << log_m;
  const size_t N = (size_t)M * R;
  const int lane = threadIdx.x & (TC - 1), wv = threadIdx.x / TC;
  const size_t c = (size_t)blockIdx.x * TC + lane;
  const bool live = c < (size_t)M;
  const int comp = blockIdx.y, item = blockIdx.z;
  const int ell = tb.ell, nl = tb.nl, k = tb.k;
  constexpr int nm = NM;  // = tb.dn_nm
  uint64_t* yw = reinterpret_cast<uint64_t*>(yp);
  for (int m = wv; m < 4 * nm; m += CW) {
    uint64_t y[R];
    if (live && m < k) {
      const LimbC L = tb.limb[ell + m];
      const uint64_t* a = accp + (((size_t)item * 2 + comp) * nl + ell + m) * N;
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = a[c + (size_t)r * M];
      sub_inv<LOGR>(ari(tb, L, ell + m, true), y, 1u);
      const uint64_t w = tb.dn_pre[2 * m], ws = tb.dn_pre[2 * m + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = mx_pack(reduce2(mul_shoup(y[r], w, ws, L.q), L.q));
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) yw[((size_t)((m >> 1) * R + r) * TC + lane) * 2 + (m & 1)] = y[r];
  }
  __syncthreads();
  const int h = lane >> 5;
  const size_t cc = (size_t)blockIdx.x * TC + (wv & 1) * 32 + (lane & 31);
  const bool clive = cc < (size_t)M;
  uint64_t* o = t2 + ((size_t)item * 2 + comp) * ell * N;
  const ulonglong2* cst = reinterpret_cast<const ulonglong2*>(tb.dn_mx);
  for (int g = (wv >> 1) + ((tgt0 >> 2) & ~(CW / 2 - 1)); 4 * g < tgt1; g += CW / 2) {
    if (4 * g + 4 <= tgt0) continue;
    const int ta = 4 * g + 2 * h, tb2 = ta + 1;
    const bool sa = clive && ta >= tgt0 && ta < tgt1;
    const bool sb = clive && tb2 >= tgt0 && tb2 < tgt1;
    int lt[4];
#pragma unroll
    for (int tau = 0; tau < 4; ++tau) lt[tau] = 4 * g + tau < ell ? 4 * g + tau : 0;
    mx_group<LOGR, true, NM>(tb, yp, cst + (size_t)g * nm * 64, lt, sa, sb, o + (size_t)lt[2 * h] * N,
                             o + (size_t)lt[2 * h + 1] * N, cc, M);
  }
}

// ---------------------------------------------------------- ModDown (K5)

// One block b of one Q limb i in [tgt0, tgt0 + ntgt) of one (item, component)
// pair ic = item*2 + c per workgroup (placed by xcd_tile):
// forward block pass of t2 (canonical), then out = (acc_Q - v) * P^-1 (canonical).
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE))) void k_moddown_blocks(DevTables tb, const uint64_t* t2,
                                                                         const uint64_t* acc, uint64_t* out,
                                                                         int tgt0, int ntgt, int ics,
                                                                         EvalIn ev) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * ntgt, ics);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R;
  const int i = tgt0 + tl.tile / R;
  const int ic = tl.item;
  const LimbC L = tb.limb[i];
  const uint32_t B0 = (uint32_t)R + b;
  const size_t boff = (size_t)b * B::M;
  const uint64_t* src = t2 + ((size_t)ic * tb.ell + i) * N + boff;
  double v[B::E];
#pragma unroll
  for (int e = 0; e < B::E; ++e) v[e] = u2d(src[B::fr_pos(tid, e)]);
  B::fwd(arf(tb, L, i, false), v, reinterpret_cast<double*>(lds), tid, B0);
  const uint64_t* a = acc + ((size_t)ic * tb.nl + i) * N + boff;
  uint64_t* o = out + ((size_t)ic * tb.ell + i) * N + boff;
  const double pinv = tb.dn_pinv_d[i];
  const int item = ic >> 1, comp = ic & 1;
  const size_t r0 = ((size_t)item * 2 * tb.ell + i) * N + boff, r1 = r0 + (size_t)tb.ell * N;
  // MODE 0: plain KeySwitch, 1: HMUL, 2: HROT (chosen once per workgroup)
  auto finish = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      const int x = B::cl_pos(tid, e);
      // |acc - v| <= 3.2q, |P^-1| <= q/2
      double w = f_mul(u2d(a[x]) - v[e], pinv, L.qd, L.qinv);
      if constexpr (MODE == 2) {  // HROT: sigma_g(c0) in component 0
        if (comp == 0) w += u2d(ev.a[r0 + galois_src((uint32_t)(boff + x), ev.galois, tb.log_n) - boff]);
      } else if constexpr (MODE == 1) {  // HMUL: this component's tensor term, a0 b0 or a0 b1 + a1 b0
        const double a0 = u2d(ev.a[r0 + x]);
        if (comp == 0)
          w += f_mul(a0, u2d(ev.b[r0 + x]), L.qd, L.qinv);
        else
          w += f_mul(a0, u2d(ev.b[r1 + x]), L.qd, L.qinv) + f_mul(u2d(ev.a[r1 + x]), u2d(ev.b[r0 + x]), L.qd, L.qinv);
      }
      o[x] = f_canon(w, L.qd, L.qinv);
    }
  };
  if (!ev.a)
    finish(std::integral_constant<int, 0>{});
  else if (!ev.galois)
    finish(std::integral_constant<int, 1>{});
  else
    finish(std::integral_constant<int, 2>{});
}

// The twiddles one block pass reads, staged in LDS: entry x in [1, M) is
// table entry ((R + b) << s) + x - 2^s with s = floor(log2 x), the twiddle of
// local stage s and group x - 2^s of block b. Stages s >= PS (the last round
// of the forward pass) are stored group-major: group (p << (s - PS)) + g at
// 2^s + (g << PS) + p. BlockNtt::fwd<true> with B0 = 1 and this table
// computes what BlockNtt::fwd computes with B0 = R + b and the global table.
template <int LOGM, int PS, class T>
__device__ __forceinline__ void stage_twiddles(T* tw, const T* table, uint32_t B0, int tid, int nthreads) {
  for (int x = tid; x < (1 << LOGM); x += nthreads) {
    if (x == 0) continue;
    const int s = 31 - __clz(x);
    const uint32_t grp = (uint32_t)(x - (1 << s));
    uint32_t pos = (uint32_t)x;
    if (s >= PS) {  // grp = (p << rho) + g
      const int rho = s - PS;
      pos = (1u << s) + ((grp & ((1u << rho) - 1)) << PS) + (grp >> rho);
    }
    tw[pos] = table[(B0 << s) + grp];
  }
}

// ModDown's last block pass with the Q-limb KeyMult of digit-parallel plans
// folded in. One block b of one Q limb i in [tgt0, tgt0 + ntgt) of one item
// per workgroup (placed by xcd_tile), all five forward block passes of the
// limb share its twiddles, staged once in LDS:
//   s_c = -NTT(t2_c) + sum_{j in [j0, j1)} ext_j * evk[j][c],
//   ext_j = d (i in D_j) or the forward block pass of ext1 slot j,
//   out_c = s_c * P^-1 (canonical).
// t2 and ext1 canonical in, |values| <= 2.2q inside. Inputs and key blocks are
// loaded before the transform that precedes their use, so that their latency
// overlaps it.
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE)), (LOGE == 3 && LOGM >= 12) ? 4 : 1) void k_moddown_km_blocks(
    DevTables tb, const uint64_t* d, const uint64_t* ext1, const uint64_t* evk, const uint64_t* t2, uint64_t* out,
    int j0, int j1, int nslots, int slot_stride, int tgt0, int ntgt, int items, EvalIn ev) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  double* ld = reinterpret_cast<double*>(lds);
  // Staged twiddles up to blocks of 2^12 (beyond, the extra LDS would leave
  // one workgroup per CU, which costs more than the table reads it saves).
  constexpr bool TWL = LOGM <= 12;
  double* tw = ld + B::LDS_WORDS;
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * ntgt, items);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R;
  const int i = tgt0 + tl.tile / R;
  const int item = tl.item;
  const LimbC L = tb.limb[i];
  const int nl = tb.nl, ell = tb.ell;
  const size_t boff = (size_t)b * B::M;
  const ArF A{L.qd, L.qinv, TWL ? tw : tb.twf_d + (size_t)i * N};
  const uint32_t B0 = TWL ? 1u : (uint32_t)(R + b);
  const int own = i / tb.alpha;  // the digit whose limbs include i: its input is d, already in NTT form
  // Loads ahead of use: always the second t2 component and the first key
  // component of a digit; with DEEP also the next digit's input and the
  // second key component (registers allow it up to blocks of 2^12).
  constexpr bool DEEP = LOGM <= 12;
  // input of digit j: d (CL layout) for the own digit, else ext1 (FR layout)
  auto load_digit = [&](int j, double* x) {
    if (j == own) {
      const uint64_t* src = d + ((size_t)item * ell + i) * N + boff;
#pragma unroll
      for (int e = 0; e < B::E; ++e) x[e] = u2d(src[B::cl_pos(tid, e)]);
    } else {
      const uint64_t* src = ext1 + (((size_t)item * nslots + (slot_stride ? j : 0)) * nl + i) * N + boff;
#pragma unroll
      for (int e = 0; e < B::E; ++e) x[e] = u2d(src[B::fr_pos(tid, e)]);
    }
  };
  double s0[B::E], s1[B::E], cur[B::E], nxt[B::E];
  {
    const uint64_t* src = t2 + (((size_t)item * 2 + 0) * ell + i) * N + boff;
#pragma unroll
    for (int e = 0; e < B::E; ++e) cur[e] = u2d(src[B::fr_pos(tid, e)]);
  }
  if constexpr (TWL) {
    stage_twiddles<LOGM, B::LAST_S0>(tw, tb.twf_d + (size_t)i * N, (uint32_t)(R + b), tid, B::T);
    __syncthreads();
  }
  {
    const uint64_t* src = t2 + (((size_t)item * 2 + 1) * ell + i) * N + boff;
#pragma unroll
    for (int e = 0; e < B::E; ++e) nxt[e] = u2d(src[B::fr_pos(tid, e)]);
  }
  fwd_opaque<B, TWL>(A, cur, ld, tid, B0);
#pragma unroll
  for (int e = 0; e < B::E; ++e) {
    s0[e] = -cur[e];
    cur[e] = nxt[e];
  }
  if (DEEP && j0 < j1) load_digit(j0, nxt);
  fwd_opaque<B, TWL>(A, cur, ld, tid, B0);
#pragma unroll
  for (int e = 0; e < B::E; ++e) s1[e] = -cur[e];
  for (int j = j0; j < j1; ++j) {
    if constexpr (DEEP) {
#pragma unroll
      for (int e = 0; e < B::E; ++e) cur[e] = nxt[e];
    }
    const uint64_t* k0 = evk + key_row(tb, j, 0, i) * N + boff;
    const uint64_t* k1 = evk + key_row(tb, j, 1, i) * N + boff;
    double w0[B::E], w1[B::E];
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      w0[e] = u2d(k0[B::cl_pos(tid, e)]);
      if constexpr (DEEP) w1[e] = u2d(k1[B::cl_pos(tid, e)]);
    }
    if constexpr (DEEP) {
      if (j + 1 < j1) load_digit(j + 1, nxt);
    } else {
      load_digit(j, cur);
    }
    if (j != own) fwd_opaque<B, TWL>(A, cur, ld, tid, B0);
    if constexpr (!DEEP) {
#pragma unroll
      for (int e = 0; e < B::E; ++e) w1[e] = u2d(k1[B::cl_pos(tid, e)]);
    }
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      s0[e] += f_mul(cur[e], w0[e], L.qd, L.qinv);
      s1[e] += f_mul(cur[e], w1[e], L.qd, L.qinv);
    }
    if (((j - j0) & 3) == 3) {
#pragma unroll
      for (int e = 0; e < B::E; ++e) {
        s0[e] = f_red(s0[e], L.qd, L.qinv);
        s1[e] = f_red(s1[e], L.qd, L.qinv);
      }
    }
  }
  const double pinv = tb.dn_pinv_d[i];
  const size_t r0 = (((size_t)item * 2 + 0) * ell + i) * N + boff, r1 = (((size_t)item * 2 + 1) * ell + i) * N + boff;
  // MODE 0: plain KeySwitch, 1: HMUL, 2: HROT (chosen once per workgroup)
  auto finish = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      const int x = B::cl_pos(tid, e);
      double v0 = f_mul(f_red(s0[e], L.qd, L.qinv), pinv, L.qd, L.qinv);
      double v1 = f_mul(f_red(s1[e], L.qd, L.qinv), pinv, L.qd, L.qinv);
      if constexpr (MODE != 0)  // |v| stays below 3q
        add_eval<MODE == 2>(L, ev, r0 + x, r1 + x, (uint32_t)(boff + x), tb.log_n, v0, v1);
      __builtin_nontemporal_store(f_canon(v0, L.qd, L.qinv), out + r0 + x);  // the result is not read again here
      __builtin_nontemporal_store(f_canon(v1, L.qd, L.qinv), out + r1 + x);
    }
  };
  if (!ev.a)
    finish(std::integral_constant<int, 0>{});
  else if (!ev.galois)
    finish(std::integral_constant<int, 1>{});
  else
    finish(std::integral_constant<int, 2>{});
}

// --------------------------------- hoisted forward passes (KS_PLAN_HOIST_FWD)

// The digit-parallel KeyMult and ModDown tail when the raised digits are
// already forward-transformed (k_ext_blocks ran on ext1 in place, canonical
// residues in natural order): every workgroup then handles one component of
// one (limb, block, item) and runs at most one transform, so a launch has
// twice the workgroups of K3 / K5 and a quarter to a third of their serial
// chain, which is what a single small ciphertext needs.

// P limbs: acc_c[t] = sum_j ext1[j][t] * evk[j][c][t] (Montgomery products,
// running sums in [0, 2q)), then the inverse block pass; stored like K3's
// finalize (accp in [0, 2q), first-round layout). Tile (P limb, block),
// item (item, component).
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE))) void k_keymult_pre(DevTables tb, const uint64_t* ext1,
                                                                      const uint64_t* evk, uint64_t* acc, int items2) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * tb.k, items2);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R;
  const int t = tb.ell + tl.tile / R;
  const int item = tl.item >> 1, c = tl.item & 1;
  const LimbC L = tb.limb[t];
  const int nl = tb.nl;
  const size_t boff = (size_t)b * B::M;
  uint64_t s[B::E];
#pragma unroll
  for (int i = 0; i < B::E; ++i) s[i] = 0;
  for (int j = 0; j < tb.ndig; ++j) {
    const uint64_t* src = ext1 + (((size_t)item * tb.ndig + j) * nl + t) * N + boff;
    const uint64_t* key = evk + key_row(tb, j, c, t) * N + boff;
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
      const int x = B::cl_pos(tid, i);
      s[i] += mont_mul(src[x], key[x], L.q, L.mont_ninv);
      s[i] = s[i] >= L.two_q ? s[i] - L.two_q : s[i];
    }
  }
#pragma unroll
  for (int i = 0; i < B::E; ++i) s[i] = reduce2(mont_mul(s[i], L.r2, L.q, L.mont_ninv), L.q);
  inv_opaque<B>(ari(tb, L, t, true), s, lds, tid, (uint32_t)R + b);
  uint64_t* a = acc + (((size_t)item * 2 + c) * nl + t) * N + boff;
#pragma unroll
  for (int i = 0; i < B::E; ++i) a[B::fr_pos(tid, i)] = s[i];
}

// Q limbs: out_c[i] = (sum_j ext_j[i] * evk[j][c][i] - NTT(t2_c)[i]) * P^-1
// with ext_j = d for the digit that owns limb i (d, or a1 b1 / sigma(c1) for
// HMUL / HROT, natural order) and the pre-transformed ext1 slot otherwise;
// HMUL / HROT add their other terms of component c. Tile (Q limb, block),
// item (item, component).
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE))) void k_moddown_pre(DevTables tb, const uint64_t* d,
                                                                      const uint64_t* ext1, const uint64_t* evk,
                                                                      const uint64_t* t2, uint64_t* out, int items2,
                                                                      EvalIn ev) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const size_t N = (size_t)1 << tb.log_n;
  const int R = (int)(N >> LOGM);
  const Tile tl = xcd_tile(R * tb.ell, items2);
  if (!tl.valid) return;
  const int tid = threadIdx.x, b = tl.tile % R;
  const int i = tl.tile / R;
  const int item = tl.item >> 1, c = tl.item & 1;
  const LimbC L = tb.limb[i];
  const int nl = tb.nl, ell = tb.ell;
  const size_t boff = (size_t)b * B::M;
  const int own = i / tb.alpha;
  double v[B::E];
  {
    const uint64_t* src = t2 + (((size_t)item * 2 + c) * ell + i) * N + boff;
#pragma unroll
    for (int e = 0; e < B::E; ++e) v[e] = u2d(src[B::fr_pos(tid, e)]);
  }
  fwd_opaque<B>(arf(tb, L, i, false), v, reinterpret_cast<double*>(lds), tid, (uint32_t)R + b);
  double sum[B::E];
#pragma unroll
  for (int e = 0; e < B::E; ++e) sum[e] = -v[e];  // |v| <= 2.2q
  for (int j = 0; j < tb.ndig; ++j) {
    const uint64_t* src = j == own ? d + ((size_t)item * ell + i) * N + boff
                                   : ext1 + (((size_t)item * tb.ndig + j) * nl + i) * N + boff;
    const uint64_t* key = evk + key_row(tb, j, c, i) * N + boff;
#pragma unroll
    for (int e = 0; e < B::E; ++e) {
      const int x = B::cl_pos(tid, e);
      sum[e] += f_mul(u2d(src[x]), u2d(key[x]), L.qd, L.qinv);  // canonical operands: within 0.875q
    }
    if ((j & 3) == 3) {  // 2.2q + 4 * 0.875q stays below 8q <= 2^53
#pragma unroll
      for (int e = 0; e < B::E; ++e) sum[e] = f_red(sum[e], L.qd, L.qinv);
    }
  }
  const double pinv = tb.dn_pinv_d[i];
  const size_t r0 = (((size_t)item * 2 + 0) * ell + i) * N + boff, r1 = (((size_t)item * 2 + 1) * ell + i) * N + boff;
  const size_t rc = c ? r1 : r0;
#pragma unroll
  for (int e = 0; e < B::E; ++e) {
    const int x = B::cl_pos(tid, e);
    double o = f_mul(f_red(sum[e], L.qd, L.qinv), pinv, L.qd, L.qinv);
    if (ev.a) {
      if (ev.galois) {  // HROT: sigma(c0) joins component 0
        if (c == 0) o += u2d(ev.a[r0 + x - (boff + x) + galois_src((uint32_t)(boff + x), ev.galois, tb.log_n)]);
      } else {  // HMUL: a0 b0 to component 0, a0 b1 + a1 b0 to component 1
        const double a0 = u2d(ev.a[r0 + x]);
        if (c == 0)
          o += f_mul(a0, u2d(ev.b[r0 + x]), L.qd, L.qinv);
        else
          o += f_mul(a0, u2d(ev.b[r1 + x]), L.qd, L.qinv) + f_mul(u2d(ev.a[r1 + x]), u2d(ev.b[r0 + x]), L.qd, L.qinv);
      }
    }
    __builtin_nontemporal_store(f_canon(o, L.qd, L.qinv), out + rc + x);
  }
}

// ------------------------------------------------------ standalone kernels

// ks_modup: forward block pass of every non-digit limb of ext (in place).
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE))) void k_ext_blocks(DevTables tb, uint64_t* ext) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int t = blockIdx.y;
  const int j = blockIdx.z % tb.ndig;
  const int lo = j * tb.alpha;
  if (t >= lo && t < lo + tb.alpha && t < tb.ell) return;  // uniform over the workgroup
  const LimbC L = tb.limb[t];
  const size_t N = (size_t)1 << tb.log_n;
  const uint32_t B0 = (uint32_t)(N >> LOGM) + b;
  uint64_t* a = ext + ((size_t)blockIdx.z * tb.nl + t) * N + (size_t)b * B::M;
  if (t < tb.ell) {
    double v[B::E];
#pragma unroll
    for (int e = 0; e < B::E; ++e) v[e] = u2d(a[B::fr_pos(tid, e)]);
    B::fwd(arf(tb, L, t, false), v, reinterpret_cast<double*>(lds), tid, B0);
#pragma unroll
    for (int e = 0; e < B::E; ++e) a[B::cl_pos(tid, e)] = f_canon(v[e], L.qd, L.qinv);
  } else {
    uint64_t v[B::E];
#pragma unroll
    for (int e = 0; e < B::E; ++e) v[e] = a[B::fr_pos(tid, e)];
    B::fwd(ari(tb, L, t, false), v, lds, tid, B0);
#pragma unroll
    for (int e = 0; e < B::E; ++e) a[B::cl_pos(tid, e)] = reduce4(v[e], L.q, L.two_q);
  }
}

// ext[item][j][t] = d[item][t] for t in D_j.
__global__ void k_copy_digits(DevTables tb, const uint64_t* d, uint64_t* ext) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int t = blockIdx.y, item = blockIdx.z;
  const int j = t / tb.alpha;
  ext[(((size_t)item * tb.ndig + j) * tb.nl + t) * N + x] = d[((size_t)item * tb.ell + t) * N + x];
}

// ks_bconv: coefficient-form conversion of one source set, one thread per
// coefficient, integer arithmetic. src [items][ns][N], dst [items][nd][N].
__global__ void k_bconv(DevTables tb, const uint64_t* src, uint64_t* dst, int set) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int u = blockIdx.y, item = blockIdx.z;
  int lo, hi, t;
  if (set < 0) {
    lo = tb.ell;
    hi = tb.nl;
    t = u;
  } else {
    lo = set * tb.alpha;
    hi = min(lo + tb.alpha, tb.ell);
    t = u < lo ? u : u + (hi - lo);
  }
  const int ns = hi - lo;
  const int nd = tb.nl - ns;
  const LimbC L = tb.limb[t];
  uint64_t z = 0;
  for (int s = 0; s < ns; ++s) {
    const int i = lo + s;
    const LimbC S = tb.limb[i];
    // y_i = x_i * [(S/s_i)^-1]_{s_i}, canonical
    const uint64_t* hinv = set < 0 ? tb.dn_hinv + 2 * s : tb.up_hinv + 2 * i;
    const uint64_t xi = src[((size_t)item * ns + s) * N + x];
    const uint64_t y = reduce2(mul_shoup(xi, hinv[0], hinv[1], S.q), S.q);
    const uint64_t* cst = set < 0 ? tb.dn_mat + 2 * ((size_t)s * tb.ell + t) : tb.up_mat + 2 * ((size_t)i * tb.nl + t);
    z += reduce2(mul_shoup(y, cst[0], cst[1], L.q), L.q);
    if ((s & 7) == 7) z = reduce2(mul_shoup(z, 1, L.red_s, L.q), L.q);
  }
  dst[((size_t)item * nd + u) * N + x] = reduce2(mul_shoup(z, 1, L.red_s, L.q), L.q);
}

// ------------------------------------------------- HMUL and HROT (element-wise)

// HMUL's tensor product over the Q limbs: for ciphertexts a, b
// [items][2][ell][N] (canonical, NTT form): t01 [items][2][ell][N] gets
// (a0 b0, a0 b1 + a1 b0) and d2 [items][ell][N] gets a1 b1, canonical.
// Grid: (ceil(N / 256), ell, items).
__global__ __launch_bounds__(256) void k_tensor(DevTables tb, const uint64_t* a, const uint64_t* b, uint64_t* t01,
                                                uint64_t* d2) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= N) return;
  const int i = blockIdx.y, item = blockIdx.z, ell = tb.ell;
  const LimbC L = tb.limb[i];
  const size_t r0 = (((size_t)item * 2 + 0) * ell + i) * N + x, r1 = (((size_t)item * 2 + 1) * ell + i) * N + x;
  const double a0 = u2d(a[r0]), a1 = u2d(a[r1]), b0 = u2d(b[r0]), b1 = u2d(b[r1]);
  t01[r0] = f_canon(f_mul(a0, b0, L.qd, L.qinv), L.qd, L.qinv);
  t01[r1] = f_canon(f_mul(a0, b1, L.qd, L.qinv) + f_mul(a1, b0, L.qd, L.qinv), L.qd, L.qinv);
  d2[((size_t)item * ell + i) * N + x] = f_canon(f_mul(a1, b1, L.qd, L.qinv), L.qd, L.qinv);
}

// The Galois automorphism x -> x^g on NTT-form limbs: slot t holds the value at
// psi^(2 brv(t) + 1), so slot t of the image is slot t' of the input with
// 2 brv(t') + 1 = g (2 brv(t) + 1) mod 2N. src and dst [rows][N] (rows =
// gridDim.y * gridDim.z, any limbs), dst must not alias src.
// Grid: (ceil(N / 256), rows per item, items).
__global__ __launch_bounds__(256) void k_automorph(int log_n, const uint64_t* src, uint64_t* dst, uint32_t g,
                                                   size_t src_item_stride, size_t dst_item_stride) {
  const uint32_t N = 1u << log_n;
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  const uint32_t e = 2u * (__brev(t) >> (32 - log_n)) + 1u;
  const uint32_t e2 = (uint32_t)(((uint64_t)g * e) & (2u * N - 1u));
  const uint32_t t2 = __brev((e2 - 1u) >> 1) >> (32 - log_n);
  const size_t row = blockIdx.y;
  dst[(size_t)blockIdx.z * dst_item_stride + row * N + t] = src[(size_t)blockIdx.z * src_item_stride + row * N + t2];
}

// out[item][c][i] += add[item][c][i] mod q_i for c < ncomp (both canonical).
// Grid: (ceil(N / 256), ncomp * ell, items).
__global__ __launch_bounds__(256) void k_add_q(DevTables tb, uint64_t* out, const uint64_t* add) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= N) return;
  const int ell = tb.ell;
  const int c = blockIdx.y / ell, i = blockIdx.y % ell, item = blockIdx.z;
  const uint64_t q = tb.limb[i].q;
  const size_t r = (((size_t)item * 2 + c) * ell + i) * N + x;
  const uint64_t v = out[r] + add[r];
  out[r] = v >= q ? v - q : v;
}

// ks_keymult: element-wise over acc [items][2][nl][N], integer arithmetic.
__global__ void k_keymult(DevTables tb, const uint64_t* ext, const uint64_t* evk, uint64_t* acc) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int t = blockIdx.y % tb.nl, c = blockIdx.y / tb.nl, item = blockIdx.z;
  const LimbC L = tb.limb[t];
  uint64_t s = 0;
  for (int j = 0; j < tb.ndig; ++j) {
    s += mont_mul(ext[(((size_t)item * tb.ndig + j) * tb.nl + t) * N + x], evk[key_row(tb, j, c, t) * N + x],
                  L.q, L.mont_ninv);
    s = s >= L.two_q ? s - L.two_q : s;
  }
  acc[(((size_t)item * 2 + c) * tb.nl + t) * N + x] = reduce2(mont_mul(s, L.r2, L.q, L.mont_ninv), L.q);
}

// ks_moddown, first step: inverse block pass of the P limbs of acc
// (canonical) into the work buffer accp (same layout), values in [0, 2q).
template <int LOGM, int LOGE>
__global__ __launch_bounds__((1 << (LOGM - LOGE))) void k_pblocks_inv(DevTables tb, const uint64_t* acc,
                                                                      uint64_t* accp) {
  using B = BlockNtt<LOGM, LOGE>;
  extern __shared__ uint64_t lds[];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int t = tb.ell + blockIdx.y;
  const int ic = blockIdx.z;
  const LimbC L = tb.limb[t];
  const size_t N = (size_t)1 << tb.log_n;
  const uint32_t B0 = (uint32_t)(N >> LOGM) + b;
  const size_t off = ((size_t)ic * tb.nl + t) * N + (size_t)b * B::M;
  uint64_t v[B::E];
#pragma unroll
  for (int e = 0; e < B::E; ++e) v[e] = acc[off + B::cl_pos(tid, e)];
  B::inv(ari(tb, L, t, true), v, lds, tid, B0);
#pragma unroll
  for (int e = 0; e < B::E; ++e) accp[off + B::fr_pos(tid, e)] = v[e];
}

// ------------------------------------------------------------ dispatching

// LDS of an MFMA column workgroup: 2 nm pairs of 16-byte digit words per row and column.
inline size_t mx_lds_bytes(int nm, int log_r) { return (size_t)nm * ((size_t)1 << log_r) * TC * 32; }

template <template <int> class F, typename... A>
hipError_t by_logr(int log_r, A... a) {
  switch (log_r) {
    case 0: return F<0>::run(a...);
    case 1: return F<1>::run(a...);
    case 2: return F<2>::run(a...);
    case 3: return F<3>::run(a...);
    case 4: return F<4>::run(a...);
    case 5: return F<5>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

// The MFMA column kernels hold 2R values per lane: at most 32 rows (at 32 rows
// with two waves per SIMD).
template <template <int> class F, typename... A>
hipError_t by_logr_mx(int log_r, A... a) {
  switch (log_r) {
    case 0: return F<0>::run(a...);
    case 1: return F<1>::run(a...);
    case 2: return F<2>::run(a...);
    case 3: return F<3>::run(a...);
    case 4: return F<4>::run(a...);
    case 5: return F<5>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

// Elements per thread of the plain block passes: 16 from blocks of 2^12 on,
// 8 below (twice the threads per block, which small transforms need to fill
// the chip: -22% on (2, 2^13, 6) with one ciphertext).
constexpr int loge_for(int logm) { return logm >= 12 ? 4 : (logm >= 6 ? 3 : (logm >= 4 ? 2 : 1)); }

// Latency variant of a block pass: 4 elements per thread (8 at blocks of
// 2^13), so that a block of 2^11 to 2^13 coefficients runs on 512 to 1024
// threads. A launch whose default configuration would leave the chip short of
// threads (a single small ciphertext) is bound by the serial chain of each
// thread and by latencies that its few waves cannot hide; halving or
// quartering the elements per thread shortens the chain and puts up to four
// waves on every SIMD that runs a block.
constexpr int loge_lat(int logm) { return logm >= 13 ? 3 : 2; }

// Whether a launch of `wgs` workgroups of blocks of 2^logm with 2^loge
// elements per thread has fewer than 2^18 threads (4 waves per SIMD over the
// 1024 SIMDs): then its latency variant runs instead.
inline bool use_lat(int logm, int loge, long wgs) {
  return logm >= 8 && logm <= 13 && loge_lat(logm) < loge && wgs * (1L << (logm - loge)) < (1L << 18);
}

template <template <int, int> class F, typename... A>
hipError_t by_logm(int log_m, long wgs, A... a) {
  switch (log_m) {
#define KS_CASE(m) \
  case m:          \
    return use_lat(m, loge_for(m), wgs) ? F<m, loge_lat(m)>::run(a...) : F<m, loge_for(m)>::run(a...);
    KS_CASE(3) KS_CASE(4) KS_CASE(5) KS_CASE(6) KS_CASE(7) KS_CASE(8) KS_CASE(9) KS_CASE(10) KS_CASE(11)
    KS_CASE(12) KS_CASE(13) KS_CASE(14)
#undef KS_CASE
    default: return hipErrorInvalidValue;
  }
}

// KeyMult keeps two accumulators per element across the digits, so its block
// passes run with 8 elements per thread up to M = 2^13 (1024 threads at 2^13)
// and 16 beyond. K5 also holds its prefetched inputs and key blocks: 8
// elements per thread up to 2^12, 16 from 2^13 on (at 1024 threads it would
// spill).
constexpr int loge_k3(int logm) { return logm >= 14 ? 4 : (logm >= 6 ? 3 : (logm >= 4 ? 2 : 1)); }
constexpr int loge_k5(int logm) { return logm >= 13 ? 4 : loge_k3(logm); }

template <template <int, int> class F, bool K5 = false, typename... A>
hipError_t by_logm_k3(int log_m, long wgs, A... a) {
  switch (log_m) {
#define KS_CASE(m)                                                                   \
  case m:                                                                            \
    return use_lat(m, K5 ? loge_k5(m) : loge_k3(m), wgs) ? F<m, loge_lat(m)>::run(a...) \
                                                         : F<m, K5 ? loge_k5(m) : loge_k3(m)>::run(a...);
    KS_CASE(3) KS_CASE(4) KS_CASE(5) KS_CASE(6) KS_CASE(7) KS_CASE(8) KS_CASE(9) KS_CASE(10) KS_CASE(11)
    KS_CASE(12) KS_CASE(13) KS_CASE(14)
#undef KS_CASE
    default: return hipErrorInvalidValue;
  }
}

dim3 col_grid(int log_m, int y, int z) {
  return dim3((unsigned)(((1 << log_m) + TC - 1) / TC), (unsigned)y, (unsigned)z);
}

template <int LOGM, int LOGE>
size_t block_lds() {
  return sizeof(uint64_t) * BlockNtt<LOGM, LOGE>::LDS_WORDS;
}

// Lets a kernel take up to the whole 160 KB of LDS as dynamic shared memory
// (done once per kernel instantiation).
template <auto Kernel>
void allow_lds() {
  static const hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)once;
}

template <int LOGR>
struct ColsFwd {
  static hipError_t run(const DevTables& tb, uint64_t* x, int first, int nl, int items, int log_m, hipStream_t s) {
    k_cols<LOGR, false><<<col_grid(log_m, nl, items), dim3(TC), 0, s>>>(tb, x, first, nl, log_m);
    return hipGetLastError();
  }
};
template <int LOGR>
struct ColsInv {
  static hipError_t run(const DevTables& tb, uint64_t* x, int first, int nl, int items, int log_m, hipStream_t s) {
    k_cols<LOGR, true><<<col_grid(log_m, nl, items), dim3(TC), 0, s>>>(tb, x, first, nl, log_m);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct BlocksFwd {
  static hipError_t run(const DevTables& tb, const uint64_t* src, uint64_t* dst, int first, int nl, int items,
                        int scale, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_blocks<LOGM, LOGE, false>>();
    k_blocks<LOGM, LOGE, false><<<dim3(xcd_grid(nl << (tb.log_n - LOGM), items)), dim3(B::T),
                                  block_lds<LOGM, LOGE>(), s>>>(tb, src, dst, first, nl, items, scale);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct BlocksInv {
  static hipError_t run(const DevTables& tb, const uint64_t* src, uint64_t* dst, int first, int nl, int items,
                        int scale, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_blocks<LOGM, LOGE, true>>();
    k_blocks<LOGM, LOGE, true><<<dim3(xcd_grid(nl << (tb.log_n - LOGM), items)), dim3(B::T),
                                 block_lds<LOGM, LOGE>(), s>>>(tb, src, dst, first, nl, items, scale);
    return hipGetLastError();
  }
};
template <int LOGR>
struct ModupCols {
  static hipError_t run(const DevTables& tb, const uint64_t* t1, uint64_t* ext1, int j0, int nj, int nslots,
                        int slot_stride, int tgt0, int tgt1, int items, int log_m, hipStream_t s) {
    allow_lds<k_modup_cols<LOGR>>();
    const size_t lds = sizeof(double) * (size_t)tb.alpha * (1 << LOGR) * TC;
    k_modup_cols<LOGR><<<col_grid(log_m, nj, items), dim3(CT), lds, s>>>(tb, t1, ext1, j0, nslots, slot_stride, tgt0,
                                                                         tgt1, log_m);
    return hipGetLastError();
  }
};
template <int LOGR, int NM>
hipError_t modup_cols_mx(const DevTables& tb, const uint64_t* t1, uint64_t* ext1, int j0, int nj, int nslots,
                         int slot_stride, int tgt0, int tgt1, int items, int log_m, hipStream_t s) {
  allow_lds<k_modup_cols_mx<LOGR, NM>>();
  k_modup_cols_mx<LOGR, NM><<<col_grid(log_m, nj, items), dim3(CT), mx_lds_bytes(NM, LOGR), s>>>(
      tb, t1, ext1, j0, nslots, slot_stride, tgt0, tgt1, log_m);
  return hipGetLastError();
}
template <int LOGR>
struct ModupColsMx {
  template <typename... A>
  static hipError_t run(const DevTables& tb, A... a) {
    switch (tb.up_nm) {
      case 1: return modup_cols_mx<LOGR, 1>(tb, a...);
      case 2: return modup_cols_mx<LOGR, 2>(tb, a...);
      case 3: return modup_cols_mx<LOGR, 3>(tb, a...);
      case 4: return modup_cols_mx<LOGR, 4>(tb, a...);
      default: return hipErrorInvalidValue;
    }
  }
};
template <int LOGM, int LOGE>
struct KeymultBlocks {
  static hipError_t run(const DevTables& tb, const uint64_t* d, const uint64_t* ext1, const uint64_t* evk,
                        uint64_t* acc, int j0, int j1, int nslots, int slot_stride, int tgt0, int tgt1, int items,
                        int accumulate, int finalize, int q_part, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    const int qend = tgt1 < tb.ell ? tgt1 : tb.ell;
    if (q_part && tgt0 < qend) {
      allow_lds<k_keymult_blocks<LOGM, LOGE, true>>();
      k_keymult_blocks<LOGM, LOGE, true><<<dim3(xcd_grid((qend - tgt0) << (tb.log_n - LOGM), items)), dim3(B::T),
                                           block_lds<LOGM, LOGE>(), s>>>(tb, d, ext1, evk, acc, j0, j1, nslots,
                                                                         slot_stride, tgt0, qend - tgt0, items,
                                                                         accumulate, finalize);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const int pbeg = tgt0 > tb.ell ? tgt0 : tb.ell;
    if (pbeg < tgt1) {
      allow_lds<k_keymult_blocks<LOGM, LOGE, false>>();
      k_keymult_blocks<LOGM, LOGE, false><<<dim3(xcd_grid((tgt1 - pbeg) << (tb.log_n - LOGM), items)), dim3(B::T),
                                            block_lds<LOGM, LOGE>(), s>>>(tb, d, ext1, evk, acc, j0, j1, nslots,
                                                                          slot_stride, pbeg, tgt1 - pbeg, items,
                                                                          accumulate, finalize);
    }
    return hipGetLastError();
  }
};
template <int LOGR>
struct ModdownCols {
  static hipError_t run(const DevTables& tb, const uint64_t* accp, uint64_t* t2, int tgt0, int tgt1, int items,
                        int log_m, hipStream_t s) {
    allow_lds<k_moddown_cols<LOGR>>();
    const size_t lds = sizeof(uint64_t) * (size_t)tb.k * (1 << LOGR) * TC;
    k_moddown_cols<LOGR><<<col_grid(log_m, 2, items), dim3(CT), lds, s>>>(tb, accp, t2, tgt0, tgt1, log_m);
    return hipGetLastError();
  }
};
template <int LOGR, int NM>
hipError_t moddown_cols_mx(const DevTables& tb, const uint64_t* accp, uint64_t* t2, int tgt0, int tgt1, int items,
                           int log_m, hipStream_t s) {
  allow_lds<k_moddown_cols_mx<LOGR, NM>>();
  k_moddown_cols_mx<LOGR, NM><<<col_grid(log_m, 2, items), dim3(CT), mx_lds_bytes(NM, LOGR), s>>>(
      tb, accp, t2, tgt0, tgt1, log_m);
  return hipGetLastError();
}
template <int LOGR>
struct ModdownColsMx {
  template <typename... A>
  static hipError_t run(const DevTables& tb, A... a) {
    switch (tb.dn_nm) {
      case 1: return moddown_cols_mx<LOGR, 1>(tb, a...);
      case 2: return moddown_cols_mx<LOGR, 2>(tb, a...);
      case 3: return moddown_cols_mx<LOGR, 3>(tb, a...);
      case 4: return moddown_cols_mx<LOGR, 4>(tb, a...);
      default: return hipErrorInvalidValue;
    }
  }
};
template <int LOGM, int LOGE>
struct ModdownBlocks {
  static hipError_t run(const DevTables& tb, const uint64_t* t2, const uint64_t* acc, uint64_t* out, int tgt0,
                        int tgt1, int items, EvalIn ev, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_moddown_blocks<LOGM, LOGE>>();
    k_moddown_blocks<LOGM, LOGE><<<dim3(xcd_grid((tgt1 - tgt0) << (tb.log_n - LOGM), items * 2)), dim3(B::T),
                                   block_lds<LOGM, LOGE>(), s>>>(tb, t2, acc, out, tgt0, tgt1 - tgt0, items * 2, ev);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct EvalBlocks {
  static hipError_t run(const DevTables& tb, EvalIn ev, uint64_t* d2, uint64_t* t1, int items, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_eval_blocks<LOGM, LOGE>>();
    k_eval_blocks<LOGM, LOGE><<<dim3(xcd_grid(tb.ell << (tb.log_n - LOGM), items)), dim3(B::T),
                                block_lds<LOGM, LOGE>(), s>>>(tb, ev, d2, t1, items);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
size_t km_lds() {
  using B = BlockNtt<LOGM, LOGE>;
  return LOGM <= 12 ? sizeof(double) * (B::LDS_WORDS + B::M) : block_lds<LOGM, LOGE>();
}
template <int LOGM, int LOGE>
struct ModdownKmBlocks {
  static hipError_t run(const DevTables& tb, const uint64_t* d, const uint64_t* ext1, const uint64_t* evk,
                        const uint64_t* t2, uint64_t* out, int j0, int j1, int nslots, int slot_stride, int tgt0,
                        int tgt1, int items, EvalIn ev, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_moddown_km_blocks<LOGM, LOGE>>();
    k_moddown_km_blocks<LOGM, LOGE><<<dim3(xcd_grid((tgt1 - tgt0) << (tb.log_n - LOGM), items)), dim3(B::T),
                                      km_lds<LOGM, LOGE>(), s>>>(tb, d, ext1, evk, t2, out, j0, j1, nslots,
                                                                    slot_stride, tgt0, tgt1 - tgt0, items, ev);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct KeymultPre {
  static hipError_t run(const DevTables& tb, const uint64_t* ext1, const uint64_t* evk, uint64_t* acc, int items,
                        hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_keymult_pre<LOGM, LOGE>>();
    k_keymult_pre<LOGM, LOGE><<<dim3(xcd_grid(tb.k << (tb.log_n - LOGM), 2 * items)), dim3(B::T),
                                block_lds<LOGM, LOGE>(), s>>>(tb, ext1, evk, acc, 2 * items);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct ModdownPre {
  static hipError_t run(const DevTables& tb, const uint64_t* d, const uint64_t* ext1, const uint64_t* evk,
                        const uint64_t* t2, uint64_t* out, int items, EvalIn ev, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_moddown_pre<LOGM, LOGE>>();
    k_moddown_pre<LOGM, LOGE><<<dim3(xcd_grid(tb.ell << (tb.log_n - LOGM), 2 * items)), dim3(B::T),
                                block_lds<LOGM, LOGE>(), s>>>(tb, d, ext1, evk, t2, out, 2 * items, ev);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct ExtBlocks {
  static hipError_t run(const DevTables& tb, uint64_t* ext, int items, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_ext_blocks<LOGM, LOGE>>();
    k_ext_blocks<LOGM, LOGE><<<dim3(1u << (tb.log_n - LOGM), tb.nl, items * tb.ndig), dim3(B::T),
                               block_lds<LOGM, LOGE>(), s>>>(tb, ext);
    return hipGetLastError();
  }
};
template <int LOGM, int LOGE>
struct PBlocksInv {
  static hipError_t run(const DevTables& tb, const uint64_t* acc, uint64_t* accp, int items, hipStream_t s) {
    using B = BlockNtt<LOGM, LOGE>;
    allow_lds<k_pblocks_inv<LOGM, LOGE>>();
    k_pblocks_inv<LOGM, LOGE><<<dim3(1u << (tb.log_n - LOGM), tb.k, items * 2), dim3(B::T),
                                block_lds<LOGM, LOGE>(), s>>>(tb, acc, accp);
    return hipGetLastError();
  }
};

}  // namespace

// ------------------------------------------------------------ launchers

// The column kernels stage count * 2^log_r values per column in LDS (64
// columns per workgroup, 8 bytes each, at most 160 KB).
int stage_cap(int count, int log_r) { return (size_t)count * ((size_t)1 << log_r) * 64 * 8 <= 160 * 1024 ? 1 : 0; }

int mx_ok(const DevTables& tb, int log_r) {
  // at most 16 sources (the partial-sum bound), 32 rows per column (registers), LDS
  return tb.up_nm <= 4 && tb.dn_nm <= 4 && log_r <= 5 && mx_lds_bytes(tb.up_nm, log_r) <= 160 * 1024 &&
         mx_lds_bytes(tb.dn_nm, log_r) <= 160 * 1024;
}

hipError_t launch_ntt(const DevTables& tb, int log_r, uint64_t* x, int first, int nlimbs, int items, hipStream_t s) {
  const int log_m = tb.log_n - log_r;
  hipError_t e = hipSuccess;
  if (log_r > 0) e = by_logr<ColsFwd>(log_r, tb, x, first, nlimbs, items, log_m, s);
  if (e != hipSuccess) return e;
  return by_logm<BlocksFwd>(log_m, (long)(nlimbs << log_r) * items, tb, (const uint64_t*)x, x, first, nlimbs, items,
                            0, s);
}

hipError_t launch_intt(const DevTables& tb, int log_r, uint64_t* x, int first, int nlimbs, int items, hipStream_t s) {
  const int log_m = tb.log_n - log_r;
  hipError_t e = by_logm<BlocksInv>(log_m, (long)(nlimbs << log_r) * items, tb, (const uint64_t*)x, x, first, nlimbs,
                                    items, log_r == 0 ? 1 : 0, s);
  if (e != hipSuccess || log_r == 0) return e;
  return by_logr<ColsInv>(log_r, tb, x, first, nlimbs, items, log_m, s);
}

hipError_t launch_intt_blocks(const DevTables& tb, int log_r, const uint64_t* src, uint64_t* dst, int nlimbs,
                              int items, hipStream_t s) {
  return by_logm<BlocksInv>(tb.log_n - log_r, (long)(nlimbs << log_r) * items, tb, src, dst, 0, nlimbs, items, 0, s);
}

hipError_t launch_eval_blocks(const DevTables& tb, int log_r, EvalIn ev, uint64_t* d2, uint64_t* t1, int items,
                              hipStream_t s) {
  return by_logm<EvalBlocks>(tb.log_n - log_r, (long)(tb.ell << log_r) * items, tb, ev, d2, t1, items, s);
}

hipError_t launch_modup_cols(const DevTables& tb, int log_r, const uint64_t* t1, uint64_t* ext1, int j0, int nj,
                             int nslots, int slot_stride, int tgt0, int tgt1, int items, int mfma, hipStream_t s) {
  if (mfma)
    return by_logr_mx<ModupColsMx>(log_r, tb, t1, ext1, j0, nj, nslots, slot_stride, tgt0, tgt1, items,
                                tb.log_n - log_r, s);
  return by_logr<ModupCols>(log_r, tb, t1, ext1, j0, nj, nslots, slot_stride, tgt0, tgt1, items, tb.log_n - log_r, s);
}

hipError_t launch_keymult_blocks(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                                 const uint64_t* evk, uint64_t* acc, int j0, int j1, int nslots, int slot_stride,
                                 int tgt0, int tgt1, int items, int accumulate, int finalize, int q_part,
                                 hipStream_t s) {
  return by_logm_k3<KeymultBlocks>(tb.log_n - log_r, (long)((tgt1 - tgt0) << log_r) * items, tb, d, ext1, evk, acc,
                                   j0, j1, nslots, slot_stride, tgt0, tgt1, items, accumulate, finalize, q_part, s);
}

hipError_t launch_moddown_km_blocks(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                                    const uint64_t* evk, const uint64_t* t2, uint64_t* out, int j0, int j1,
                                    int nslots, int slot_stride, int tgt0, int tgt1, int items, EvalIn ev,
                                    hipStream_t s) {
  return by_logm_k3<ModdownKmBlocks, true>(tb.log_n - log_r, (long)((tgt1 - tgt0) << log_r) * items, tb, d, ext1, evk,
                                           t2, out, j0, j1, nslots, slot_stride, tgt0, tgt1, items, ev, s);
}

hipError_t launch_moddown_cols(const DevTables& tb, int log_r, const uint64_t* accp, uint64_t* t2, int tgt0,
                               int tgt1, int items, int mfma, hipStream_t s) {
  if (mfma) return by_logr_mx<ModdownColsMx>(log_r, tb, accp, t2, tgt0, tgt1, items, tb.log_n - log_r, s);
  return by_logr<ModdownCols>(log_r, tb, accp, t2, tgt0, tgt1, items, tb.log_n - log_r, s);
}

hipError_t launch_moddown_blocks(const DevTables& tb, int log_r, const uint64_t* t2, const uint64_t* acc,
                                 uint64_t* out, int tgt0, int tgt1, int items, EvalIn ev, hipStream_t s) {
  return by_logm<ModdownBlocks>(tb.log_n - log_r, (long)((tgt1 - tgt0) << log_r) * items * 2, tb, t2, acc, out, tgt0,
                                tgt1, items, ev, s);
}

hipError_t launch_ext_blocks(const DevTables& tb, int log_r, uint64_t* ext, int items, hipStream_t s) {
  return by_logm<ExtBlocks>(tb.log_n - log_r, (long)(tb.nl << log_r) * items * tb.ndig, tb, ext, items, s);
}

hipError_t launch_keymult_pre(const DevTables& tb, int log_r, const uint64_t* ext1, const uint64_t* evk,
                              uint64_t* acc, int items, hipStream_t s) {
  return by_logm<KeymultPre>(tb.log_n - log_r, (long)(tb.k << log_r) * items * 2, tb, ext1, evk, acc, items, s);
}

hipError_t launch_moddown_pre(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                              const uint64_t* evk, const uint64_t* t2, uint64_t* out, int items, EvalIn ev,
                              hipStream_t s) {
  return by_logm<ModdownPre>(tb.log_n - log_r, (long)(tb.ell << log_r) * items * 2, tb, d, ext1, evk, t2, out, items,
                             ev, s);
}

hipError_t launch_pblocks_inv(const DevTables& tb, int log_r, const uint64_t* acc, uint64_t* accp, int items,
                              hipStream_t s) {
  return by_logm<PBlocksInv>(tb.log_n - log_r, (long)(tb.k << log_r) * items * 2, tb, acc, accp, items, s);
}

hipError_t launch_copy_digits(const DevTables& tb, const uint64_t* d, uint64_t* ext, int items, hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_copy_digits<<<dim3((n + 255) / 256, tb.ell, items), dim3(256), 0, s>>>(tb, d, ext);
  return hipGetLastError();
}

hipError_t launch_bconv(const DevTables& tb, const uint64_t* src, int set, uint64_t* dst, int items, hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  int nd;
  if (set < 0) {
    nd = tb.ell;
  } else {
    const int lo = set * tb.alpha;
    const int hi = lo + tb.alpha < tb.ell ? lo + tb.alpha : tb.ell;
    nd = tb.nl - (hi - lo);
  }
  k_bconv<<<dim3((n + 255) / 256, nd, items), dim3(256), 0, s>>>(tb, src, dst, set);
  return hipGetLastError();
}

hipError_t launch_tensor(const DevTables& tb, const uint64_t* a, const uint64_t* b, uint64_t* t01, uint64_t* d2,
                         int items, hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_tensor<<<dim3((n + 255) / 256, tb.ell, items), dim3(256), 0, s>>>(tb, a, b, t01, d2);
  return hipGetLastError();
}

hipError_t launch_automorph(const DevTables& tb, const uint64_t* src, uint64_t* dst, int rows, size_t src_item_stride,
                            size_t dst_item_stride, uint32_t g, int items, hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_automorph<<<dim3((n + 255) / 256, rows, items), dim3(256), 0, s>>>(tb.log_n, src, dst, g, src_item_stride,
                                                                       dst_item_stride);
  return hipGetLastError();
}

hipError_t launch_add_q(const DevTables& tb, uint64_t* out, const uint64_t* add, int ncomp, int items,
                        hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_add_q<<<dim3((n + 255) / 256, ncomp * tb.ell, items), dim3(256), 0, s>>>(tb, out, add);
  return hipGetLastError();
}

// Throughput probe of the three modular products the kernels are built
// from. Every thread runs MM_CHAINS independent chains of `iters` dependent
// products by a fixed operand (enough chains to hide the latency of one
// product), then folds its chains into sink[thread] so that no product is
// dead code. kind 0: FP64 product of the Q primes (f_mul); 1: Shoup product
// of the P primes (mul_shoup); 2: Montgomery product (mont_mul).
constexpr int MM_CHAINS = MODMUL_CHAINS;

template <int KIND>
__global__ __launch_bounds__(256) void k_modmul_rate(int iters, uint64_t q, uint64_t w, uint64_t ws, uint64_t ninv,
                                                     double qd, double qinv, double wd, uint64_t* sink) {
  const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
  if (KIND == 0) {
    double a[MM_CHAINS];
#pragma unroll
    for (int c = 0; c < MM_CHAINS; ++c) a[c] = (double)(tid * MM_CHAINS + c + 1);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < MM_CHAINS; ++c) a[c] = f_mul(a[c], wd, qd, qinv);
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < MM_CHAINS; ++c) acc = f_red(acc + a[c], qd, qinv);
    sink[tid] = f_canon(acc, qd, qinv);
  } else {
    uint64_t a[MM_CHAINS];
#pragma unroll
    for (int c = 0; c < MM_CHAINS; ++c) a[c] = (uint64_t)(tid * MM_CHAINS + c + 1);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < MM_CHAINS; ++c) a[c] = KIND == 1 ? mul_shoup(a[c], w, ws, q) : mont_mul(a[c], w, q, ninv);
    }
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < MM_CHAINS; ++c) acc ^= a[c];
    sink[tid] = acc;
  }
}

hipError_t launch_modmul_rate(int kind, int blocks, int iters, uint64_t q, uint64_t w, uint64_t ws, uint64_t ninv,
                              uint64_t* sink, hipStream_t s) {
  const double qd = (double)q, qinv = 1.0 / qd;
  // the fixed operand in balanced form for the FP64 product
  const double wd = w > q / 2 ? (double)w - qd : (double)w;
  switch (kind) {
    case 0: k_modmul_rate<0><<<dim3(blocks), dim3(256), 0, s>>>(iters, q, w, ws, ninv, qd, qinv, wd, sink); break;
    case 1: k_modmul_rate<1><<<dim3(blocks), dim3(256), 0, s>>>(iters, q, w, ws, ninv, qd, qinv, wd, sink); break;
    case 2: k_modmul_rate<2><<<dim3(blocks), dim3(256), 0, s>>>(iters, q, w, ws, ninv, qd, qinv, wd, sink); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Input check of the debug build: flag[0] = 1 if some word of x is not a
// canonical residue of its row's prime. x holds `items` blocks of item_words
// words; row r of an item (N words at offset r * N) belongs to limb
// row_limb[r] of the extended basis (negative: a row the call does not read).
// Grid: (ceil(N / 256), rows, items).
__global__ __launch_bounds__(256) void k_check_rows(DevTables tb, const uint64_t* x, const int* row_limb,
                                                    size_t item_words, int* flag) {
  const size_t N = (size_t)1 << tb.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int limb = row_limb[blockIdx.y];
  if (c >= N || limb < 0) return;
  if (x[(size_t)blockIdx.z * item_words + (size_t)blockIdx.y * N + c] >= tb.limb[limb].q) *flag = 1;
}

hipError_t launch_check_rows(const DevTables& tb, const uint64_t* x, const int* row_limb, int rows, int items,
                             size_t item_words, int* flag, hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_check_rows<<<dim3((n + 255) / 256, rows, items), dim3(256), 0, s>>>(tb, x, row_limb, item_words, flag);
  return hipGetLastError();
}

// HBM copy probe: dst[i] = src[i] for `words` 64-bit words, each thread
// moving 8 (kind 0) or 16 bytes (kind 1) per access with a grid-stride loop,
// stores cached or non-temporal (nt). The practical streaming ceiling of the
// access widths the kernels use.
template <int WIDE, bool NT>
__global__ __launch_bounds__(256) void k_copy_rate(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                   size_t words) {
  const size_t stride = (size_t)gridDim.x * 256;
  if (WIDE) {
    const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(src);
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(dst);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words / 2; i += stride) {
      const ulonglong2 v = s2[i];
      if (NT) {
        __builtin_nontemporal_store(v.x, &d2[i].x);
        __builtin_nontemporal_store(v.y, &d2[i].y);
      } else {
        d2[i] = v;
      }
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += stride) {
      if (NT)
        __builtin_nontemporal_store(src[i], dst + i);
      else
        dst[i] = src[i];
    }
  }
}

hipError_t launch_copy_rate(int kind, int nt, int blocks, const uint64_t* src, uint64_t* dst, size_t words,
                            hipStream_t s) {
  const dim3 g(blocks), t(256);
  if (kind == 0 && !nt) k_copy_rate<0, false><<<g, t, 0, s>>>(src, dst, words);
  else if (kind == 0) k_copy_rate<0, true><<<g, t, 0, s>>>(src, dst, words);
  else if (kind == 1 && !nt) k_copy_rate<1, false><<<g, t, 0, s>>>(src, dst, words);
  else if (kind == 1) k_copy_rate<1, true><<<g, t, 0, s>>>(src, dst, words);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_keymult(const DevTables& tb, const uint64_t* ext, const uint64_t* evk, uint64_t* acc, int items,
                          hipStream_t s) {
  const unsigned n = 1u << tb.log_n;
  k_keymult<<<dim3((n + 255) / 256, 2 * tb.nl, items), dim3(256), 0, s>>>(tb, ext, evk, acc);
  return hipGetLastError();
}

}  // namespace ks
