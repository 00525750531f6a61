// Host launchers of the KeySwitch kernels (ks_kernels.hip). Every launcher
// only enqueues on stream `s` and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ks_device.hpp"

namespace ks {

// Nonzero when the column kernels can stage `count` source limbs of 2^log_r
// rows each in LDS.
int stage_cap(int count, int log_r);
// Nonzero when the int8-MFMA BConv column kernels support these parameters
// at this NTT split.
int mx_ok(const DevTables& tb, int log_r);

// Two-pass transforms of x [items][nlimbs][N], limb r over prime first + r.
hipError_t launch_ntt(const DevTables& tb, int log_r, uint64_t* x, int first, int nlimbs, int items, hipStream_t s);
hipError_t launch_intt(const DevTables& tb, int log_r, uint64_t* x, int first, int nlimbs, int items, hipStream_t s);
// Inverse block pass only (stages log_n-1 .. log_r) of src [items][nlimbs][N] over primes 0..nlimbs-1.
hipError_t launch_intt_blocks(const DevTables& tb, int log_r, const uint64_t* src, uint64_t* dst, int nlimbs,
                              int items, hipStream_t s);
// mfma: BConv on the int8 matrix cores (requires mx_ok) instead of FP64 / integer products.
hipError_t launch_modup_cols(const DevTables& tb, int log_r, const uint64_t* t1, uint64_t* ext1, int j0, int nj,
                             int nslots, int slot_stride, int tgt0, int tgt1, int items, int mfma, hipStream_t s);
// KeyMult over targets [tgt0, tgt1): one kernel for the Q limbs (skipped when
// q_part is 0) and one for the P limbs.
hipError_t launch_keymult_blocks(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                                 const uint64_t* evk, uint64_t* acc, int j0, int j1, int nslots, int slot_stride,
                                 int tgt0, int tgt1, int items, int accumulate, int finalize, int q_part,
                                 hipStream_t s);
// ModDown's last block pass with the Q-limb KeyMult of digits [j0, j1) folded in.
hipError_t launch_moddown_km_blocks(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                                    const uint64_t* evk, const uint64_t* t2, uint64_t* out, int j0, int j1,
                                    int nslots, int slot_stride, int tgt0, int tgt1, int items, EvalIn ev,
                                    hipStream_t s);
hipError_t launch_moddown_cols(const DevTables& tb, int log_r, const uint64_t* accp, uint64_t* t2, int tgt0,
                               int tgt1, int items, int mfma, hipStream_t s);
// ev (HMUL / HROT, ev.a null for a plain KeySwitch): adds the tensor terms or sigma_g(c0) to out.
hipError_t launch_moddown_blocks(const DevTables& tb, int log_r, const uint64_t* t2, const uint64_t* acc,
                                 uint64_t* out, int tgt0, int tgt1, int items, EvalIn ev, hipStream_t s);
// First pass of a fused HMUL / HROT: d2 = a1 b1 or sigma_g(c1), and its inverse block pass t1.
hipError_t launch_eval_blocks(const DevTables& tb, int log_r, EvalIn ev, uint64_t* d2, uint64_t* t1, int items,
                              hipStream_t s);
hipError_t launch_ext_blocks(const DevTables& tb, int log_r, uint64_t* ext, int items, hipStream_t s);
// Hoisted forward passes (ext1 [items][ndig][nl][N] already forward-transformed by launch_ext_blocks):
// the P-limb KeyMult and inverse block pass into acc (as K3's finalize), one component per workgroup;
hipError_t launch_keymult_pre(const DevTables& tb, int log_r, const uint64_t* ext1, const uint64_t* evk,
                              uint64_t* acc, int items, hipStream_t s);
// and ModDown's last pass over the Q limbs with their KeyMult (as K5), one component per workgroup.
hipError_t launch_moddown_pre(const DevTables& tb, int log_r, const uint64_t* d, const uint64_t* ext1,
                              const uint64_t* evk, const uint64_t* t2, uint64_t* out, int items, EvalIn ev,
                              hipStream_t s);
hipError_t launch_pblocks_inv(const DevTables& tb, int log_r, const uint64_t* acc, uint64_t* accp, int items,
                              hipStream_t s);
hipError_t launch_copy_digits(const DevTables& tb, const uint64_t* d, uint64_t* ext, int items, hipStream_t s);
hipError_t launch_bconv(const DevTables& tb, const uint64_t* src, int set, uint64_t* dst, int items, hipStream_t s);
// HMUL tensor product: t01 [items][2][ell][N] = (a0 b0, a0 b1 + a1 b0), d2 [items][ell][N] = a1 b1.
hipError_t launch_tensor(const DevTables& tb, const uint64_t* a, const uint64_t* b, uint64_t* t01, uint64_t* d2,
                         int items, hipStream_t s);
// Galois automorphism x -> x^g of `rows` NTT-form limbs per item (strides in words).
hipError_t launch_automorph(const DevTables& tb, const uint64_t* src, uint64_t* dst, int rows, size_t src_item_stride,
                            size_t dst_item_stride, uint32_t g, int items, hipStream_t s);
// out [items][2][ell][N] += add (same layout) for components c < ncomp, mod q_i.
hipError_t launch_add_q(const DevTables& tb, uint64_t* out, const uint64_t* add, int ncomp, int items,
                        hipStream_t s);
hipError_t launch_keymult(const DevTables& tb, const uint64_t* ext, const uint64_t* evk, uint64_t* acc, int items,
                          hipStream_t s);
// Modular-product throughput probe: blocks x 256 threads x MODMUL_CHAINS chains x
// iters products of kind 0 (FP64, modulus q < 2^50), 1 (Shoup) or 2
// (Montgomery); sink [blocks * 256].
constexpr int MODMUL_CHAINS = 8;
// Debug-build input check: *flag = 1 if a word of x [items][rows][N] (item
// stride item_words) is not below the prime of its row (row_limb[r] < 0: skip).
hipError_t launch_check_rows(const DevTables& tb, const uint64_t* x, const int* row_limb, int rows, int items,
                             size_t item_words, int* flag, hipStream_t s);
// HBM copy probe: dst = src over `words` words (even for kind 1), 8 (kind 0)
// or 16 (kind 1) bytes per access, non-temporal stores when nt != 0.
hipError_t launch_copy_rate(int kind, int nt, int blocks, const uint64_t* src, uint64_t* dst, size_t words,
                            hipStream_t s);
hipError_t launch_modmul_rate(int kind, int blocks, int iters, uint64_t q, uint64_t w, uint64_t ws, uint64_t ninv,
                              uint64_t* sink, hipStream_t s);

}  // namespace ks
