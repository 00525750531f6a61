// C ABI of libks (include/ks.h): parameter handles, argument checks, and the
// plan executor that orders the kernels of one KeySwitch by dataflow
// (DSOB, DPOB, DSOC, DPOC of the paper's classification, or the staged
// ModUp / KeyMult / ModDown sequence).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ks.h"
#include "ks_host.hpp"
#include "ks_kernels.hpp"

struct ks_params {
  ks::HostParams hp;
  ks::DevTables tb;
  void* blob = nullptr;
  int device = 0;
  // Second stream of KS_PLAN_SPLIT_STREAMS plans, with the fork and join
  // events; `split` serialises their use by concurrent callers.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex split;
  // Debug build only: device flag word followed by the row table of the input
  // check (see dbg_check), serialised by dbg_mu.
  int* dbg = nullptr;
  std::mutex dbg_mu;
};

// Scratch memory of ks_keyswitch_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends. In host code
// `scratch` names a host-side stand-in, not device memory; the device address
// of each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) when the first parameter handle is made there, and
// only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[KS_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_hip_error = "none";

// Launch trace of the calling thread (ks_trace_begin / ks_trace_end).
struct Trace {
  bool active = false;
  hipEvent_t* events = nullptr;
  int cap = 0, n = 0;
  unsigned mask = 0;
  std::vector<int> kinds;
};
thread_local Trace g_trace;

// Runs one launch, bracketed by trace events when tracing is on for `kind`.
template <class F>
hipError_t traced(int kind, hipStream_t s, F&& launch) {
  Trace& t = g_trace;
  const bool rec = t.active && ((t.mask >> kind) & 1u) && t.n < t.cap;
  if (rec) {
    const hipError_t e = hipEventRecord(t.events[2 * t.n], s);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = launch();
  if (rec && e == hipSuccess) {
    const hipError_t e2 = hipEventRecord(t.events[2 * t.n + 1], s);
    if (e2 != hipSuccess) return e2;
    t.kinds.push_back(kind);
    ++t.n;
  }
  return e;
}

int hip_fail(hipError_t e) {
  g_hip_error = hipGetErrorName(e);
  return KS_EHIP;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

int check_ptr(const void* p) {
  if (!p) return KS_ENULL;
  if (!aligned(p)) return KS_EALIGN;
  return KS_OK;
}

// Default NTT split: blocks of 2^12 coefficients from N = 2^14 up, 2^10 below
// (enough workgroups for a single ciphertext), one pass for tiny N.
int default_log_r(int log_n) {
  if (log_n >= 14) return log_n - 12;
  return log_n >= 10 ? log_n - 10 : 0;
}

// Plan validity for these parameters: the NTT split must be compiled and the
// BConv sources of the column kernels must fit their register staging.
int resolve_plan(const ks_params* p, const ks_plan* in, ks_plan& out) {
  if (in) {
    out = *in;
  } else {
    out = ks_plan{KS_DPOB, 1, -1, 0, 0};
  }
  if (out.flags & ~(KS_PLAN_MFMA_BCONV | KS_PLAN_SPLIT_STREAMS | KS_PLAN_HOIST_FWD)) return KS_EUNSUP;
  if ((out.flags & KS_PLAN_HOIST_FWD) && out.dataflow != KS_DPOB) return KS_EUNSUP;
  if (out.batch_tile < 0) return KS_EUNSUP;
  if (out.dataflow < KS_DSOB || out.dataflow > KS_STAGED) return KS_EUNSUP;
  if (out.log_r < 0) {
    // the default split, or the nearest smaller one whose column kernels can
    // stage the digit's and P's limbs (large alpha), or a larger one if the
    // blocks would otherwise exceed 2^14 coefficients
    const int d = default_log_r(p->hp.log_n);
    auto fits = [&](int r) {
      const int m = p->hp.log_n - r;
      return m >= 3 && m <= 14 && ks::stage_cap(p->hp.alpha, r) && ks::stage_cap(p->hp.k, r);
    };
    out.log_r = d;
    for (int r = d; r >= 0; --r)
      if (fits(r)) { out.log_r = r; break; }
    if (!fits(out.log_r))
      for (int r = d + 1; r <= 5; ++r)
        if (fits(r)) { out.log_r = r; break; }
  }
  const int log_m = p->hp.log_n - out.log_r;
  if (out.log_r > 5 || log_m < 3 || log_m > 14) return KS_EUNSUP;
  if (ks::stage_cap(p->hp.alpha, out.log_r) == 0 || ks::stage_cap(p->hp.k, out.log_r) == 0) return KS_EUNSUP;
  if ((out.flags & KS_PLAN_MFMA_BCONV) && !ks::mx_ok(p->tb, out.log_r)) return KS_EUNSUP;
  if (out.dataflow == KS_DSOC || out.dataflow == KS_DPOC) {
    if (out.chunks < 1 || out.chunks > 64 || out.chunks > p->hp.ell) return KS_EUNSUP;
  } else {
    out.chunks = 1;
  }
  return KS_OK;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Layout {
  size_t t1, ext1, acc, t2, accp, ext, total;
  int nslots;
};

// Workspace layout of one KeySwitch under `plan` for `batch` items.
Layout layout(const ks_params* p, int batch, const ks_plan& plan) {
  const size_t N = p->hp.n, B = (size_t)batch, W = sizeof(uint64_t);
  const size_t ell = p->hp.ell, nl = p->hp.nl;
  Layout L{};
  if (plan.dataflow == KS_STAGED) {
    // [ext][acc][scratch = max(t1, accp + t2)]
    L.ext = 0;
    L.acc = up256(B * p->hp.ndig * nl * N * W);
    const size_t scratch = L.acc + up256(B * 2 * nl * N * W);
    L.t1 = scratch;
    L.accp = scratch;
    L.t2 = scratch + up256(B * 2 * nl * N * W);
    L.total = std::max(L.t1 + up256(B * ell * N * W), L.t2 + up256(B * 2 * ell * N * W));
    return L;
  }
  const bool dp = plan.dataflow == KS_DPOB || plan.dataflow == KS_DPOC;
  L.nslots = dp ? p->hp.ndig : 1;
  L.t1 = 0;
  L.ext1 = L.t1 + up256(B * ell * N * W);
  L.acc = L.ext1 + up256(B * L.nslots * nl * N * W);
  L.t2 = L.acc + up256(B * 2 * nl * N * W);
  L.total = L.t2 + up256(B * 2 * ell * N * W);
  return L;
}

// A split plan runs items [0, b0) on the caller's stream and [b0, batch) on
// the handle's second stream, each with its own workspace.
bool split_batch(const ks_plan& plan, int batch, int& b0) {
  b0 = batch / 2;
  return (plan.flags & KS_PLAN_SPLIT_STREAMS) && batch >= 2;
}

// Items per pass: a tiled plan runs the batch in consecutive tiles of
// batch_tile items, each with the workspace (and cache footprint) of a tile.
int tile_of(const ks_plan& plan, int batch) {
  return (plan.batch_tile > 0 && plan.batch_tile < batch) ? plan.batch_tile : batch;
}

size_t workspace_total(const ks_params* p, int batch, const ks_plan& plan) {
  int b0;
  batch = tile_of(plan, batch);
  if (split_batch(plan, batch, b0)) return layout(p, b0, plan).total + layout(p, batch - b0, plan).total;
  return layout(p, batch, plan).total;
}

void chunk_range(int n, int c, int i, int& a, int& b) {
  a = (int)((long)n * i / c);
  b = (int)((long)n * (i + 1) / c);
}

#define KS_TRY(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

// Rows of the input check: one limb index per row of an input (negative: a
// row the call does not read), for the debug build's canonical-input test.
size_t dbg_rows_max(const ks::HostParams& hp, const ks::DevTables& tb) {
  return std::max({(size_t)hp.ndig * 2 * tb.evk_nl, (size_t)hp.ndig * hp.nl, (size_t)2 * hp.nl});
}

#ifdef KS_DEBUG_CHECKS
thread_local bool g_capturing = false;

// The Q limbs of a polynomial, `copies` times ([copies][ell] rows).
std::vector<int> rows_q(const ks_params* p, int copies) {
  std::vector<int> r;
  for (int c = 0; c < copies; ++c)
    for (int i = 0; i < p->hp.ell; ++i) r.push_back(i);
  return r;
}
// Limbs first .. first + n - 1 of the extended basis, `copies` times.
std::vector<int> rows_range(int first, int n, int copies) {
  std::vector<int> r;
  for (int c = 0; c < copies; ++c)
    for (int i = 0; i < n; ++i) r.push_back(first + i);
  return r;
}
// The key rows a call reads: digits 0 .. ndig-1 of [ndig_top][2][evk_nl][N];
// row t < ell is limb t, row evk_p0 + m is P limb m, other rows are unread.
std::vector<int> rows_key(const ks_params* p) {
  const ks::DevTables& tb = p->tb;
  std::vector<int> r;
  for (int j = 0; j < p->hp.ndig; ++j)
    for (int c = 0; c < 2; ++c)
      for (int row = 0; row < tb.evk_nl; ++row)
        r.push_back(row < tb.ell ? row : (row >= tb.evk_p0 ? tb.ell + (row - tb.evk_p0) : -1));
  return r;
}

// Debug build: KS_EINVAL unless every word x reads is a canonical residue of
// its row's prime. Enqueues a read-only check on s and waits for it (so a
// debug build synchronises on every call); skipped while a graph is captured.
int dbg_check(const ks_params* p, const uint64_t* x, const std::vector<int>& rows, int items, hipStream_t s) {
  if (g_capturing || items <= 0 || rows.empty()) return KS_OK;
  std::lock_guard<std::mutex> lock(const_cast<ks_params*>(p)->dbg_mu);
  const int zero = 0;
  int flag = 0;
  KS_TRY(hipMemcpyAsync(p->dbg + 1, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice, s));
  KS_TRY(hipMemcpyAsync(p->dbg, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  KS_TRY(ks::launch_check_rows(p->tb, x, p->dbg + 1, (int)rows.size(), items, rows.size() * p->hp.n, p->dbg, s));
  KS_TRY(hipMemcpyAsync(&flag, p->dbg, sizeof(int), hipMemcpyDeviceToHost, s));
  KS_TRY(hipStreamSynchronize(s));
  return flag ? KS_EINVAL : KS_OK;
}
#define KS_DEBUG_CHECK(expr)              \
  do {                                    \
    const int rc_ = (expr);               \
    if (rc_ != KS_OK) return rc_;         \
  } while (0)
#else
#define KS_DEBUG_CHECK(expr) \
  do {                       \
  } while (0)
#endif

int run_modup(const ks_params* p, const ks_plan& plan, const uint64_t* d, uint64_t* ext, int batch, uint64_t* t1,
              hipStream_t s) {
  const ks::DevTables& tb = p->tb;
  const int mx = plan.flags & KS_PLAN_MFMA_BCONV;
  KS_TRY(traced(KS_K_INTT_D, s, [&] { return ks::launch_intt_blocks(tb, plan.log_r, d, t1, tb.ell, batch, s); }));
  KS_TRY(traced(KS_K_MODUP_COLS, s, [&] { return ks::launch_modup_cols(tb, plan.log_r, t1, ext, 0, tb.ndig, tb.ndig, 1, 0, tb.nl, batch, mx, s); }));
  KS_TRY(traced(KS_K_EXT_BLOCKS, s, [&] { return ks::launch_ext_blocks(tb, plan.log_r, ext, batch, s); }));
  KS_TRY(traced(KS_K_COPY_DIGITS, s, [&] { return ks::launch_copy_digits(tb, d, ext, batch, s); }));
  return KS_OK;
}

int run_moddown(const ks_params* p, const ks_plan& plan, const uint64_t* acc, uint64_t* out, int batch,
                uint64_t* accp, uint64_t* t2, hipStream_t s) {
  const ks::DevTables& tb = p->tb;
  const int mx = plan.flags & KS_PLAN_MFMA_BCONV;
  KS_TRY(traced(KS_K_PBLOCKS_INV, s, [&] { return ks::launch_pblocks_inv(tb, plan.log_r, acc, accp, batch, s); }));
  KS_TRY(traced(KS_K_MODDOWN_COLS, s, [&] { return ks::launch_moddown_cols(tb, plan.log_r, accp, t2, 0, tb.ell, batch, mx, s); }));
  KS_TRY(traced(KS_K_MODDOWN_BLOCKS, s, [&] {
    return ks::launch_moddown_blocks(tb, plan.log_r, t2, acc, out, 0, tb.ell, batch, ks::EvalIn{}, s);
  }));
  return KS_OK;
}

// Number of kernels launch_keymult_blocks starts for targets [a, b).
int km_kernels(const ks::DevTables& tb, int a, int b, bool q_part) {
  const int qend = std::min(b, tb.ell), pbeg = std::max(a, tb.ell);
  return ((q_part && a < qend) ? 1 : 0) + (pbeg < b ? 1 : 0);
}

// The fused plans. Digit-serial plans (DSOB, DSOC) accumulate acc over
// digits and finish with ModDown's block pass; digit-parallel plans (DPOB,
// DPOC) run KeyMult only for the P limbs up front (their sum feeds ModDown's
// BConv) and fold the Q-limb KeyMult into ModDown's last block pass, so acc_Q
// never goes through memory.
//
// HMUL / HROT (ev.a not null): d is a workspace buffer that the first pass
// fills with a1 b1 or sigma_g(c1), and ModDown's last pass adds the other
// tensor terms (a0 b0, a0 b1 + a1 b0) or sigma_g(c0) to its output, so the
// operation costs no kernel beyond the KeySwitch's own.
int run_fused(const ks_params* p, const ks_plan& plan, const uint64_t* d, const uint64_t* evk, uint64_t* out,
              int batch, char* ws, hipStream_t s, int* launches, ks::EvalIn ev = ks::EvalIn{}) {
  const ks::DevTables& tb = p->tb;
  const Layout L = layout(p, batch, plan);
  uint64_t* t1 = reinterpret_cast<uint64_t*>(ws + L.t1);
  uint64_t* ext1 = reinterpret_cast<uint64_t*>(ws + L.ext1);
  uint64_t* acc = reinterpret_cast<uint64_t*>(ws + L.acc);
  uint64_t* t2 = reinterpret_cast<uint64_t*>(ws + L.t2);
  const bool dp = plan.dataflow == KS_DPOB || plan.dataflow == KS_DPOC;
  const int mx = plan.flags & KS_PLAN_MFMA_BCONV;
  const int c = plan.chunks;
  int count = 0;
  const bool run = launches == nullptr;
  if (run && ev.a)
    KS_TRY(traced(KS_K_INTT_D, s, [&] {
      return ks::launch_eval_blocks(tb, plan.log_r, ev, const_cast<uint64_t*>(d), t1, batch, s);
    }));
  else if (run)
    KS_TRY(traced(KS_K_INTT_D, s, [&] { return ks::launch_intt_blocks(tb, plan.log_r, d, t1, tb.ell, batch, s); }));
  ++count;
  if (plan.flags & KS_PLAN_HOIST_FWD) {
    // DPOB with the raised digits' forward block pass in a launch of its own,
    // then KeyMult and ModDown's tail one component per workgroup
    if (run) {
      KS_TRY(traced(KS_K_MODUP_COLS, s, [&] {
        return ks::launch_modup_cols(tb, plan.log_r, t1, ext1, 0, tb.ndig, L.nslots, 1, 0, tb.nl, batch, mx, s);
      }));
      KS_TRY(traced(KS_K_EXT_BLOCKS, s, [&] { return ks::launch_ext_blocks(tb, plan.log_r, ext1, batch, s); }));
      KS_TRY(traced(KS_K_KEYMULT_BLOCKS, s, [&] {
        return ks::launch_keymult_pre(tb, plan.log_r, ext1, evk, acc, batch, s);
      }));
      KS_TRY(traced(KS_K_MODDOWN_COLS, s, [&] {
        return ks::launch_moddown_cols(tb, plan.log_r, acc, t2, 0, tb.ell, batch, mx, s);
      }));
      KS_TRY(traced(KS_K_MODDOWN_BLOCKS, s, [&] {
        return ks::launch_moddown_pre(tb, plan.log_r, d, ext1, evk, t2, out, batch, ev, s);
      }));
    }
    if (launches) *launches = count + 5;
    return KS_OK;
  }
  for (int ci = 0; ci < c; ++ci) {
    int a, b;
    chunk_range(tb.nl, c, ci, a, b);
    if (a == b) continue;
    if (dp) {
      if (run) {
        KS_TRY(traced(KS_K_MODUP_COLS, s, [&] {
          return ks::launch_modup_cols(tb, plan.log_r, t1, ext1, 0, tb.ndig, L.nslots, 1, a, b, batch, mx, s);
        }));
        if (km_kernels(tb, a, b, false))
          KS_TRY(traced(KS_K_KEYMULT_BLOCKS, s, [&] {
            return ks::launch_keymult_blocks(tb, plan.log_r, d, ext1, evk, acc, 0, tb.ndig, L.nslots, 1, a, b, batch,
                                             0, 1, 0, s);
          }));
      }
      count += 1 + km_kernels(tb, a, b, false);
    } else {
      for (int j = 0; j < tb.ndig; ++j) {
        if (run) {
          KS_TRY(traced(KS_K_MODUP_COLS, s, [&] {
            return ks::launch_modup_cols(tb, plan.log_r, t1, ext1, j, 1, 1, 0, a, b, batch, mx, s);
          }));
          KS_TRY(traced(KS_K_KEYMULT_BLOCKS, s, [&] {
            return ks::launch_keymult_blocks(tb, plan.log_r, d, ext1, evk, acc, j, j + 1, 1, 0, a, b, batch, j > 0,
                                             j == tb.ndig - 1, 1, s);
          }));
        }
        count += 1 + km_kernels(tb, a, b, true);
      }
    }
  }
  for (int ci = 0; ci < c; ++ci) {
    int a, b;
    chunk_range(tb.ell, c, ci, a, b);
    if (a == b) continue;
    if (run) {
      KS_TRY(traced(KS_K_MODDOWN_COLS, s, [&] { return ks::launch_moddown_cols(tb, plan.log_r, acc, t2, a, b, batch, mx, s); }));
      if (dp)
        KS_TRY(traced(KS_K_MODDOWN_BLOCKS, s, [&] {
          return ks::launch_moddown_km_blocks(tb, plan.log_r, d, ext1, evk, t2, out, 0, tb.ndig, L.nslots, 1, a, b,
                                              batch, ev, s);
        }));
      else
        KS_TRY(traced(KS_K_MODDOWN_BLOCKS, s, [&] {
          return ks::launch_moddown_blocks(tb, plan.log_r, t2, acc, out, a, b, batch, ev, s);
        }));
    }
    count += 2;
  }
  if (launches) *launches = count;
  return KS_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array; `device` must be current.
hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = static_cast<char*>(ptr);
  return hipSuccess;
}

char* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace

extern "C" {

// Uploads the tables of p->hp and creates the handle's stream and events;
// destroys p on failure.
static int finish_params(ks_params* p, ks_params** out) {
  std::vector<uint64_t> blob;
  ks::build_tables(p->hp, blob, p->tb);
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = scratch_init(p->device);
  if (e == hipSuccess) e = hipMalloc(&p->blob, blob.size() * sizeof(uint64_t));
#ifdef KS_DEBUG_CHECKS
  if (e == hipSuccess) e = hipMalloc(&p->dbg, sizeof(int) * (1 + dbg_rows_max(p->hp, p->tb)));
#endif
  if (e == hipSuccess) e = hipMemcpy(p->blob, blob.data(), blob.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p->blob) (void)hipFree(p->blob);
    if (p->dbg) (void)hipFree(p->dbg);
    delete p;
    return e == hipErrorOutOfMemory ? KS_ENOMEM : hip_fail(e);
  }
  const uintptr_t base = reinterpret_cast<uintptr_t>(p->blob);
  auto rebase = [base](auto& ptr) {
    ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + reinterpret_cast<uintptr_t>(ptr));
  };
  rebase(p->tb.limb);
  rebase(p->tb.twf);
  rebase(p->tb.twi);
  rebase(p->tb.up_pre);
  rebase(p->tb.up_mat);
  rebase(p->tb.dn_pre);
  rebase(p->tb.dn_mat);
  rebase(p->tb.dn_pinv);
  rebase(p->tb.up_hinv);
  rebase(p->tb.dn_hinv);
  rebase(p->tb.up_mx);
  rebase(p->tb.dn_mx);
  rebase(p->tb.twf_d);
  rebase(p->tb.twi_d);
  rebase(p->tb.up_pre_d);
  rebase(p->tb.up_mat_d);
  rebase(p->tb.dn_mat_d);
  rebase(p->tb.dn_pinv_d);
  e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    ks_params_destroy(p);
    return hip_fail(e);
  }
  *out = p;
  return KS_OK;
}

int ks_params_create(int dnum, int log_n, int ell, ks_params** out) {
  if (!out) return KS_ENULL;
  *out = nullptr;
  if (log_n < 3 || log_n > 17 || ell < 1 || dnum < 1 || dnum > ell) return KS_EINVAL;
  const int alpha = (ell + dnum - 1) / dnum;
  if (ell + alpha > KS_MAX_LIMBS) return KS_EINVAL;
  ks_params* p = new (std::nothrow) ks_params;
  if (!p) return KS_ENOMEM;
  if (!ks::derive_params(dnum, log_n, ell, p->hp)) {
    delete p;
    return KS_EINVAL;
  }
  return finish_params(p, out);
}

int ks_params_at_level(const ks_params* top, int level, ks_params** out) {
  if (!top || !out) return KS_ENULL;
  *out = nullptr;
  if (level < 1 || level > top->hp.ell) return KS_EINVAL;
  ks_params* p = new (std::nothrow) ks_params;
  if (!p) return KS_ENOMEM;
  if (!ks::level_params(top->hp, level, p->hp)) {
    delete p;
    return KS_EINVAL;
  }
  return finish_params(p, out);
}

void ks_params_destroy(ks_params* p) {
  if (!p) return;
  if (p->side) (void)hipStreamDestroy(p->side);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->join) (void)hipEventDestroy(p->join);
  if (p->blob) (void)hipFree(p->blob);
  if (p->dbg) (void)hipFree(p->dbg);
  delete p;
}

int ks_params_info(const ks_params* p, ks_info* info) {
  if (!p || !info) return KS_ENULL;
  std::memset(info, 0, sizeof(*info));
  info->n = (int)p->hp.n;
  info->log_n = p->hp.log_n;
  info->ell = p->hp.ell;
  info->k = p->hp.k;
  info->alpha = p->hp.alpha;
  info->dnum = p->hp.dnum;
  info->ndig = p->hp.ndig;
  info->key_ell = p->hp.key_ell;
  for (int t = 0; t < p->hp.nl; ++t) {
    info->moduli[t] = p->hp.mod[t];
    info->psi[t] = p->hp.psi[t];
  }
  return KS_OK;
}

int ks_default_plan(const ks_params* p, int batch, ks_plan* plan) {
  if (!p || !plan) return KS_ENULL;
  if (batch < 0) return KS_EINVAL;
  return resolve_plan(p, nullptr, *plan);
}

int ks_workspace_bytes(const ks_params* p, int batch, const ks_plan* plan, size_t* bytes) {
  if (!p || !bytes) return KS_ENULL;
  if (batch < 0) return KS_EINVAL;
  ks_plan pl;
  const int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  *bytes = workspace_total(p, batch, pl);
  return KS_OK;
}

int ks_launch_count(const ks_params* p, int batch, const ks_plan* plan) {
  if (!p) return KS_ENULL;
  ks_plan pl;
  const int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  if (batch == 0) return 0;
  int n = 0;
  run_fused(p, pl, nullptr, nullptr, nullptr, batch, nullptr, nullptr, &n);
  const int per_pass = pl.dataflow == KS_STAGED ? 4 + 1 + 3 : n;
  const int tile = tile_of(pl, batch);
  int total = 0;
  for (int t0 = 0; t0 < batch; t0 += tile) {
    int b0;
    total += (split_batch(pl, std::min(tile, batch - t0), b0) ? 2 : 1) * per_pass;
  }
  return total;
}

// The items of a batch times `per_item` grid rows must fit one 16-bit grid
// dimension of the column kernels; the product is taken in 64 bits.
static bool batch_fits(int batch, int per_item) {
  return batch >= 0 && (int64_t)batch * (int64_t)per_item <= 65535;
}

// One call touches at most 2^31 coefficients per extended-basis array
// (batch * (ell + k) * N), so that every flattened work-item index of its
// launches fits in 31 bits.
static bool coeffs_fit(const ks_params* p, int batch, int limbs) {
  return (int64_t)batch * (int64_t)limbs * (int64_t)p->hp.n <= (int64_t(1) << 31);
}

static int check_limbs(const ks_params* p, int first, int n_limbs, int batch) {
  if (first < 0 || n_limbs < 0 || first + n_limbs > p->hp.nl || batch < 0) return KS_EINVAL;
  if (!batch_fits(batch, std::max(1, n_limbs)) || !coeffs_fit(p, batch, n_limbs)) return KS_EINVAL;
  return KS_OK;
}

int ks_ntt(const ks_params* p, uint64_t* x, int basis_first, int n_limbs, int batch, void* stream) {
  if (!p) return KS_ENULL;
  int rc = check_limbs(p, basis_first, n_limbs, batch);
  if (rc != KS_OK) return rc;
  if (n_limbs == 0 || batch == 0) return KS_OK;
  if ((rc = check_ptr(x)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, x, rows_range(basis_first, n_limbs, 1), batch, (hipStream_t)stream));
  KS_TRY(traced(KS_K_NTT, (hipStream_t)stream, [&] { return ks::launch_ntt(p->tb, default_log_r(p->hp.log_n), x, basis_first, n_limbs, batch, (hipStream_t)stream); }));
  return KS_OK;
}

int ks_intt(const ks_params* p, uint64_t* x, int basis_first, int n_limbs, int batch, void* stream) {
  if (!p) return KS_ENULL;
  int rc = check_limbs(p, basis_first, n_limbs, batch);
  if (rc != KS_OK) return rc;
  if (n_limbs == 0 || batch == 0) return KS_OK;
  if ((rc = check_ptr(x)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, x, rows_range(basis_first, n_limbs, 1), batch, (hipStream_t)stream));
  KS_TRY(traced(KS_K_NTT, (hipStream_t)stream, [&] { return ks::launch_intt(p->tb, default_log_r(p->hp.log_n), x, basis_first, n_limbs, batch, (hipStream_t)stream); }));
  return KS_OK;
}

int ks_bconv(const ks_params* p, const uint64_t* src, int src_set, uint64_t* dst, int batch, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, 1) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  if (src_set != KS_SET_P && (src_set < 0 || src_set >= p->hp.ndig)) return KS_EINVAL;
  if (batch == 0) return KS_OK;
  int rc;
  if ((rc = check_ptr(src)) != KS_OK || (rc = check_ptr(dst)) != KS_OK) return rc;
#ifdef KS_DEBUG_CHECKS
  {
    const int lo = src_set == KS_SET_P ? p->hp.ell : src_set * p->hp.alpha;
    const int ns = src_set == KS_SET_P ? p->hp.k : std::min(lo + p->hp.alpha, p->hp.ell) - lo;
    KS_DEBUG_CHECK(dbg_check(p, src, rows_range(lo, ns, 1), batch, (hipStream_t)stream));
  }
#endif
  KS_TRY(traced(KS_K_BCONV, (hipStream_t)stream, [&] { return ks::launch_bconv(p->tb, src, src_set, dst, batch, (hipStream_t)stream); }));
  return KS_OK;
}

int ks_modup(const ks_params* p, const uint64_t* d, uint64_t* ext, int batch, void* ws, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, p->hp.ndig) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  if (batch == 0) return KS_OK;
  int rc;
  if ((rc = check_ptr(d)) != KS_OK || (rc = check_ptr(ext)) != KS_OK || (rc = check_ptr(ws)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, d, rows_q(p, 1), batch, (hipStream_t)stream));
  ks_plan pl;
  const ks_plan staged{KS_STAGED, 1, -1, 0, 0};
  if ((rc = resolve_plan(p, &staged, pl)) != KS_OK) return rc;
  return run_modup(p, pl, d, ext, batch, reinterpret_cast<uint64_t*>(ws), (hipStream_t)stream);
}

int ks_keymult(const ks_params* p, const uint64_t* ext, const uint64_t* evk, uint64_t* acc, int batch,
               void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, 1) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  if (batch == 0) return KS_OK;
  int rc;
  if ((rc = check_ptr(ext)) != KS_OK || (rc = check_ptr(evk)) != KS_OK || (rc = check_ptr(acc)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, ext, rows_range(0, p->hp.nl, p->hp.ndig), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, evk, rows_key(p), 1, (hipStream_t)stream));
  KS_TRY(traced(KS_K_KEYMULT, (hipStream_t)stream, [&] { return ks::launch_keymult(p->tb, ext, evk, acc, batch, (hipStream_t)stream); }));
  return KS_OK;
}

int ks_moddown(const ks_params* p, const uint64_t* acc, uint64_t* out, int batch, void* ws, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, 2) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  if (batch == 0) return KS_OK;
  int rc;
  if ((rc = check_ptr(acc)) != KS_OK || (rc = check_ptr(out)) != KS_OK || (rc = check_ptr(ws)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, acc, rows_range(0, p->hp.nl, 2), batch, (hipStream_t)stream));
  ks_plan pl;
  const ks_plan staged{KS_STAGED, 1, -1, 0, 0};
  if ((rc = resolve_plan(p, &staged, pl)) != KS_OK) return rc;
  const size_t accp_bytes = up256((size_t)batch * 2 * p->hp.nl * p->hp.n * sizeof(uint64_t));
  uint64_t* accp = reinterpret_cast<uint64_t*>(ws);
  uint64_t* t2 = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ws) + accp_bytes);
  return run_moddown(p, pl, acc, out, batch, accp, t2, (hipStream_t)stream);
}

// One KeySwitch of `batch` items on stream s with workspace ws (no split);
// with ev.a (fused plans only) the HMUL or HROT of ev, d its workspace buffer.
static int keyswitch_on(const ks_params* p, const ks_plan& pl, const uint64_t* d, const uint64_t* evk, uint64_t* out,
                        int batch, char* ws, hipStream_t s, ks::EvalIn ev) {
  if (pl.dataflow == KS_STAGED) {
    const Layout L = layout(p, batch, pl);
    uint64_t* ext = reinterpret_cast<uint64_t*>(ws + L.ext);
    uint64_t* acc = reinterpret_cast<uint64_t*>(ws + L.acc);
    int rc;
    if ((rc = run_modup(p, pl, d, ext, batch, reinterpret_cast<uint64_t*>(ws + L.t1), s)) != KS_OK) return rc;
    KS_TRY(traced(KS_K_KEYMULT, s, [&] { return ks::launch_keymult(p->tb, ext, evk, acc, batch, s); }));
    return run_moddown(p, pl, acc, out, batch, reinterpret_cast<uint64_t*>(ws + L.accp),
                       reinterpret_cast<uint64_t*>(ws + L.t2), s);
  }
  return run_fused(p, pl, d, evk, out, batch, ws, s, nullptr, ev);
}

// keyswitch_on, or for a split plan its two halves on the two streams.
static int keyswitch_pass(const ks_params* p, const ks_plan& pl, const uint64_t* d, const uint64_t* evk,
                          uint64_t* out, int batch, char* w, hipStream_t s, ks::EvalIn ev) {
  int b0, rc;
  if (!split_batch(pl, batch, b0)) return keyswitch_on(p, pl, d, evk, out, batch, w, s, ev);
  // Items [b0, batch) on the second stream, after everything already on s;
  // s then waits for them, so the call still completes in stream order on s.
  const size_t N = p->hp.n, ell = p->hp.ell;
  const size_t ws0 = layout(p, b0, pl).total;
  const size_t ct = (size_t)b0 * 2 * ell * N;
  std::lock_guard<std::mutex> lock(const_cast<ks_params*>(p)->split);
  KS_TRY(hipEventRecord(p->fork, s));
  KS_TRY(hipStreamWaitEvent(p->side, p->fork, 0));
  const ks::EvalIn ev1{ev.a ? ev.a + ct : nullptr, ev.b ? ev.b + ct : nullptr, ev.galois};
  if ((rc = keyswitch_on(p, pl, d + (size_t)b0 * ell * N, evk, out + ct, batch - b0, w + ws0, p->side, ev1)) !=
      KS_OK)
    return rc;
  KS_TRY(hipEventRecord(p->join, p->side));
  if ((rc = keyswitch_on(p, pl, d, evk, out, b0, w, s, ev)) != KS_OK) return rc;
  KS_TRY(hipStreamWaitEvent(s, p->join, 0));
  return KS_OK;
}

// The batch in passes of batch_tile items (one pass without tiling), one
// after another in stream order on s, each reusing the workspace.
static int keyswitch_any(const ks_params* p, const ks_plan& pl, const uint64_t* d, const uint64_t* evk,
                         uint64_t* out, int batch, char* w, hipStream_t s, ks::EvalIn ev = ks::EvalIn{}) {
  const int tile = tile_of(pl, batch);
  const size_t N = p->hp.n, ell = p->hp.ell;
  for (int t0 = 0; t0 < batch; t0 += tile) {
    const size_t ct = (size_t)t0 * 2 * ell * N;
    const ks::EvalIn evt{ev.a ? ev.a + ct : nullptr, ev.b ? ev.b + ct : nullptr, ev.galois};
    const int rc = keyswitch_pass(p, pl, d + (size_t)t0 * ell * N, evk, out + ct, std::min(tile, batch - t0), w, s, evt);
    if (rc != KS_OK) return rc;
  }
  return KS_OK;
}

int ks_keyswitch(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                 const ks_plan* plan, void* ws, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, std::max(2, p->hp.ndig)) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  ks_plan pl;
  int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  if (batch == 0) return KS_OK;
  if ((rc = check_ptr(d)) != KS_OK || (rc = check_ptr(evk)) != KS_OK || (rc = check_ptr(out)) != KS_OK ||
      (rc = check_ptr(ws)) != KS_OK)
    return rc;
  KS_DEBUG_CHECK(dbg_check(p, d, rows_q(p, 1), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, evk, rows_key(p), 1, (hipStream_t)stream));
  return keyswitch_any(p, pl, d, evk, out, batch, reinterpret_cast<char*>(ws), (hipStream_t)stream);
}

int ks_keyswitch_noalloc(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                         const ks_plan* plan, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, std::max(2, p->hp.ndig)) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  ks_plan pl;
  int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  if (batch == 0) return KS_OK;
  if ((rc = check_ptr(d)) != KS_OK || (rc = check_ptr(evk)) != KS_OK || (rc = check_ptr(out)) != KS_OK) return rc;
  if (workspace_total(p, batch, pl) > KS_NOALLOC_SCRATCH_BYTES) return KS_ETOOBIG;
  KS_DEBUG_CHECK(dbg_check(p, d, rows_q(p, 1), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, evk, rows_key(p), 1, (hipStream_t)stream));
  char* ws = scratch_of(p->device);
  if (!ws) return hip_fail(hipErrorInvalidSymbol);
  // every workspace word the kernels read is written earlier in the same call,
  // so the previous call's contents need no clearing
  return keyswitch_any(p, pl, d, evk, out, batch, ws, (hipStream_t)stream);
}

// HMUL and HROT: element-wise pre-pass into the workspace, the KeySwitch of
// one component straight into `out`, then the other part added to `out`
// (under a fused plan the pre-pass and the add are folded into the
// KeySwitch's first and last passes instead).
// Workspace: [t01: B*2*ell*N][d: B*ell*N][KeySwitch workspace].
static size_t eval_extra(const ks_params* p, int batch) {
  return up256((size_t)batch * 3 * p->hp.ell * p->hp.n * sizeof(uint64_t));
}

int ks_eval_workspace_bytes(const ks_params* p, int batch, const ks_plan* plan, size_t* bytes) {
  if (!p || !bytes) return KS_ENULL;
  size_t ks = 0;
  const int rc = ks_workspace_bytes(p, batch, plan, &ks);
  if (rc != KS_OK) return rc;
  *bytes = eval_extra(p, batch) + ks;
  return KS_OK;
}

static int eval_check(const ks_params* p, const void* x, const void* y, const uint64_t* evk, const uint64_t* out,
                      void* ws) {
  int rc;
  if ((rc = check_ptr(x)) != KS_OK || (y && (rc = check_ptr(y)) != KS_OK) || (rc = check_ptr(evk)) != KS_OK ||
      (rc = check_ptr(out)) != KS_OK || (rc = check_ptr(ws)) != KS_OK)
    return rc;
  return KS_OK;
}

int ks_hmul(const ks_params* p, const uint64_t* a, const uint64_t* b, const uint64_t* evk, uint64_t* out, int batch,
            const ks_plan* plan, void* ws, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, std::max(2, p->hp.ndig)) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  ks_plan pl;
  int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  if (batch == 0) return KS_OK;
  if ((rc = eval_check(p, a, b, evk, out, ws)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, a, rows_q(p, 2), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, b, rows_q(p, 2), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, evk, rows_key(p), 1, (hipStream_t)stream));
  hipStream_t s = (hipStream_t)stream;
  const size_t LN = (size_t)p->hp.ell * p->hp.n;
  uint64_t* t01 = reinterpret_cast<uint64_t*>(ws);
  uint64_t* d2 = t01 + (size_t)batch * 2 * LN;
  char* ksws = reinterpret_cast<char*>(ws) + eval_extra(p, batch);
  if (pl.dataflow != KS_STAGED)  // the tensor product fused into the KeySwitch's first and last passes
    return keyswitch_any(p, pl, d2, evk, out, batch, ksws, s, ks::EvalIn{a, b, 0u});
  KS_TRY(traced(KS_K_EVAL, s, [&] { return ks::launch_tensor(p->tb, a, b, t01, d2, batch, s); }));
  if ((rc = keyswitch_any(p, pl, d2, evk, out, batch, ksws, s)) != KS_OK) return rc;
  KS_TRY(traced(KS_K_EVAL, s, [&] { return ks::launch_add_q(p->tb, out, t01, 2, batch, s); }));
  return KS_OK;
}

int ks_hrot(const ks_params* p, const uint64_t* ct, int galois, const uint64_t* evk, uint64_t* out, int batch,
            const ks_plan* plan, void* ws, void* stream) {
  if (!p) return KS_ENULL;
  if (!batch_fits(batch, std::max(2, p->hp.ndig)) || !coeffs_fit(p, batch, p->hp.nl)) return KS_EINVAL;
  if (galois <= 0 || (galois & 1) == 0 || (size_t)galois >= 2 * p->hp.n) return KS_EINVAL;
  ks_plan pl;
  int rc = resolve_plan(p, plan, pl);
  if (rc != KS_OK) return rc;
  if (batch == 0) return KS_OK;
  if ((rc = eval_check(p, ct, nullptr, evk, out, ws)) != KS_OK) return rc;
  KS_DEBUG_CHECK(dbg_check(p, ct, rows_q(p, 2), batch, (hipStream_t)stream));
  KS_DEBUG_CHECK(dbg_check(p, evk, rows_key(p), 1, (hipStream_t)stream));
  hipStream_t s = (hipStream_t)stream;
  const size_t LN = (size_t)p->hp.ell * p->hp.n;
  uint64_t* t01 = reinterpret_cast<uint64_t*>(ws);  // sigma(c0) in component 0
  uint64_t* d = t01 + (size_t)batch * 2 * LN;        // sigma(c1)
  char* ksws = reinterpret_cast<char*>(ws) + eval_extra(p, batch);
  if (pl.dataflow != KS_STAGED)  // sigma_g fused into the KeySwitch's first and last passes
    return keyswitch_any(p, pl, d, evk, out, batch, ksws, s, ks::EvalIn{ct, nullptr, (uint32_t)galois});
  const int ell = p->hp.ell;
  KS_TRY(traced(KS_K_EVAL, s, [&] {
    return ks::launch_automorph(p->tb, ct, t01, ell, 2 * LN, 2 * LN, (uint32_t)galois, batch, s);
  }));
  KS_TRY(traced(KS_K_EVAL, s, [&] {
    return ks::launch_automorph(p->tb, ct + LN, d, ell, 2 * LN, LN, (uint32_t)galois, batch, s);
  }));
  if ((rc = keyswitch_any(p, pl, d, evk, out, batch, ksws, s)) != KS_OK) return rc;
  KS_TRY(traced(KS_K_EVAL, s, [&] { return ks::launch_add_q(p->tb, out, t01, 1, batch, s); }));
  return KS_OK;
}

int ks_modmul_rate(const ks_params* p, int kind, int blocks, int iters, uint64_t* sink, void* stream) {
  if (!p) return KS_ENULL;
  if (kind < 0 || kind > 2 || blocks < 1 || blocks > (1 << 20) || iters < 1) return KS_EINVAL;
  int rc;
  if ((rc = check_ptr(sink)) != KS_OK) return rc;
  // the FP64 product on the first Q prime, the integer products on the first P prime
  const uint64_t q = p->hp.mod[kind == 0 ? 0 : p->hp.ell];
  const uint64_t w = q / 3 + 1;
  KS_TRY(ks::launch_modmul_rate(kind, blocks, iters, q, w, ks::host_shoup(w, q), ks::host_mont_neg_inv(q), sink,
                                (hipStream_t)stream));
  return KS_OK;
}

int ks_modmul_chains(void) { return ks::MODMUL_CHAINS; }

int ks_copy_rate(int kind, int nt, int blocks, const uint64_t* src, uint64_t* dst, size_t words, void* stream) {
  if (kind < 0 || kind > 1 || blocks < 1 || blocks > (1 << 20) || (kind == 1 && (words & 1))) return KS_EINVAL;
  if (words == 0) return KS_OK;
  int rc;
  if ((rc = check_ptr(src)) != KS_OK || (rc = check_ptr(dst)) != KS_OK) return rc;
  KS_TRY(ks::launch_copy_rate(kind, nt, blocks, src, dst, words, (hipStream_t)stream));
  return KS_OK;
}

const char* ks_strerror(int code) {
  switch (code) {
    case KS_OK: return "ok";
    case KS_EINVAL: return "invalid argument";
    case KS_ENULL: return "null pointer";
    case KS_EALIGN: return "pointer not 256-byte aligned";
    case KS_ENOMEM: return "out of memory";
    case KS_EUNSUP: return "plan not supported for these parameters";
    case KS_EHIP: return "HIP error";
    case KS_ETOOBIG: return "workspace larger than the static scratch of ks_keyswitch_noalloc (KS_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown error";
  }
}

const char* ks_last_hip_error(void) { return g_hip_error.c_str(); }

struct ks_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int ks_graph_create(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                    const ks_plan* plan, void* ws, void* stream, ks_graph** graph) {
  if (!p || !graph) return KS_ENULL;
  *graph = nullptr;
  if (!stream) return KS_ENULL;  // the legacy null stream cannot be captured
  if (batch < 1) return KS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // one eager call: validates the arguments and sets per-kernel attributes
  int rc = ks_keyswitch(p, d, evk, out, batch, plan, ws, stream);
  if (rc != KS_OK) return rc;
  ks_graph* g = new (std::nothrow) ks_graph;
  if (!g) return KS_ENOMEM;
  Trace saved = g_trace;
  g_trace = Trace{};
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
#ifdef KS_DEBUG_CHECKS
    g_capturing = true;  // the eager call above checked the inputs; a capture cannot wait on the device
#endif
    rc = ks_keyswitch(p, d, evk, out, batch, plan, ws, stream);
#ifdef KS_DEBUG_CHECKS
    g_capturing = false;
#endif
    hipGraph_t captured = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &captured);
    g->graph = captured;
    if (rc == KS_OK && e2 != hipSuccess) e = e2;
  }
  g_trace = saved;
  if (e == hipSuccess && rc == KS_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess || rc != KS_OK) {
    ks_graph_destroy(g);
    return rc != KS_OK ? rc : hip_fail(e);
  }
  *graph = g;
  return KS_OK;
}

int ks_graph_launch(ks_graph* graph, void* stream) {
  if (!graph || !graph->exec) return KS_ENULL;
  const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
  return e == hipSuccess ? KS_OK : hip_fail(e);
}

void ks_graph_destroy(ks_graph* graph) {
  if (!graph) return;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
}

int ks_trace_begin(void** events, int capacity, unsigned kind_mask) {
  if (!events && capacity > 0) return KS_ENULL;
  if (capacity < 0) return KS_EINVAL;
  Trace& t = g_trace;
  t.active = true;
  t.events = reinterpret_cast<hipEvent_t*>(events);
  t.cap = capacity;
  t.n = 0;
  t.mask = kind_mask;
  t.kinds.clear();
  return KS_OK;
}

int ks_trace_end(int* kinds, int capacity) {
  Trace& t = g_trace;
  if (!t.active) return 0;
  const int n = t.n;
  if (kinds)
    for (int i = 0; i < n && i < capacity; ++i) kinds[i] = t.kinds[i];
  t = Trace{};
  return n;
}

}  // extern "C"
