// Host-side parameter derivation and the device-resident constant tables of
// one (dnum, N, ell) parameter set.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "ks_device.hpp"

namespace ks {

struct HostParams {
  int dnum = 0, log_n = 0, ell = 0, k = 0, alpha = 0, ndig = 0, nl = 0;
  int key_ell = 0;  // Q limbs of the evaluation key (the top level's ell)
  size_t n = 0;
  std::vector<uint64_t> mod;  // q_0..q_{ell-1}, p_0..p_{k-1}
  std::vector<uint64_t> psi;  // smallest primitive 2N-th root per prime
};

// Fills `hp` from (dnum, log_n, ell); returns false if no valid set exists.
bool derive_params(int dnum, int log_n, int ell, HostParams& hp);

// The set at level `level` (1 <= level <= top.ell): Q cut to its first
// `level` primes, P, k and alpha kept, digits cut at `level`.
bool level_params(const HostParams& top, int level, HostParams& hp);

// Builds every table (twiddles, BConv constants, per-limb constants) in one
// host buffer laid out as the device expects; `dev` receives offsets relative
// to the start of that buffer (rebased after upload).
void build_tables(const HostParams& hp, std::vector<uint64_t>& blob, DevTables& offsets);

uint64_t host_mulmod(uint64_t a, uint64_t b, uint64_t m);
uint64_t host_powmod(uint64_t a, uint64_t e, uint64_t m);
uint64_t host_shoup(uint64_t w, uint64_t q);       // floor(w * 2^64 / q)
uint64_t host_mont_neg_inv(uint64_t q);            // -q^-1 mod 2^64

}  // namespace ks
