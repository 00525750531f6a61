/*
 * ks.h - C ABI of the MI355X (gfx950) CKKS hybrid KeySwitch library (libks.so).
 *
 * KeySwitch turns a polynomial d, given over the RNS basis Q = q_0..q_{ell-1}
 * in NTT form, into a pair (out_0, out_1) over Q such that
 * out_0 + out_1*s2 ~ d*s, given an evaluation key from s to s2 (Background
 * section of the paper, "KeySwitch" subsection, and its Fig. 1):
 *   ModUp   : split d into dnum digits of alpha limbs; raise each digit to the
 *             basis PQ by iNTT -> BConv -> NTT;
 *   KeyMult : multiply each raised digit by its key pair and sum over digits;
 *   ModDown : bring the sum back to Q by iNTT -> BConv -> NTT, subtract, and
 *             multiply by P^-1.
 * The order of the work (digit-serial or digit-parallel, output bulk or
 * chunked: the dataflow classification of the paper's Qualitative Analysis
 * section, Table III) is chosen by a ks_plan; every plan gives bit-identical
 * results.
 *
 * Conventions shared by every call:
 *   - Parameters: Q holds ell primes q < 2^50 and P holds k = alpha primes
 *     p < 2^60, all = 1 (mod 2N), the largest such primes in descending order;
 *     alpha = ceil(ell/dnum); digit j holds Q limbs [j*alpha, min((j+1)*alpha, ell)),
 *     and there are ndig = ceil(ell/alpha) digits. The extended basis is
 *     q_0..q_{ell-1}, p_0..p_{k-1} (limb index 0..ell+k-1).
 *   - Transform: NTT(a)[t] = sum_i a_i psi^(i*(2*brv(t)+1)) mod q with psi the
 *     smallest primitive 2N-th root of unity mod q (negacyclic ring
 *     Z_q[x]/(x^N+1), bit-reversed evaluation order). INTT is its inverse,
 *     including the factor N^-1.
 *   - BConv is the fast conversion without overflow correction:
 *     z_t = sum_i [x_i * (S/s_i)^-1]_{s_i} * (S/s_i) mod t.
 *   - Data: canonical residues in [0, modulus) stored as uint64, limb-major,
 *     coefficient index fastest. Every data pointer is a device pointer owned
 *     by the caller and aligned to 256 bytes; the library never frees it.
 *     Inputs that are not canonical residues give unspecified (but in-bounds)
 *     results in libks.so. The debug build libks_debug.so (same kernels and
 *     symbols) first checks every input word a call reads against its
 *     limb's prime and returns KS_EINVAL, with nothing else enqueued, if one
 *     is not below it; that check waits for the device, so the debug build
 *     synchronises on every call (a graph it captures skips the check).
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream). Every call only enqueues work on it and returns without
 *     synchronising; enqueued work may be captured into a HIP graph.
 *   - Errors: every int-returning call returns KS_OK (0) or a negative code;
 *     nothing is enqueued when a call fails. No exception crosses the ABI.
 *   - Batch sizes: batch >= 0 (0 enqueues nothing); the items of a batch map
 *     to one grid dimension of the column kernels, so batch * max(2, ndig)
 *     <= 65535 for ks_keyswitch, ks_hmul and ks_hrot, batch * ndig <= 65535
 *     for ks_modup, 2 * batch for ks_moddown, batch <= 65535 for ks_bconv
 *     and ks_keymult, batch * n_limbs <= 65535 for ks_ntt and ks_intt; and
 *     one call covers at most 2^31 coefficients per extended-basis array,
 *     batch * (ell + k) * N <= 2^31 (batch * n_limbs * N for ks_ntt and
 *     ks_intt), e.g. 260 items at (8, 2^17, 56). Every product is formed in
 *     64 bits; KS_EINVAL beyond, before anything is enqueued. Larger batches
 *     are split by the caller into several calls.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KS_OK 0
#define KS_EINVAL -1  /* a size or parameter is out of range */
#define KS_ENULL -2   /* a required pointer is NULL */
#define KS_EALIGN -3  /* a data pointer is not 256-byte aligned */
#define KS_ENOMEM -4  /* the library could not allocate its tables */
#define KS_EUNSUP -5  /* the plan is not valid for these parameters */
#define KS_EHIP -6    /* a HIP call failed; ks_last_hip_error() tells which */
#define KS_ETOOBIG -7 /* ks_keyswitch_noalloc: the workspace exceeds KS_NOALLOC_SCRATCH_BYTES */

#define KS_MAX_LIMBS 128 /* ell + k */
#define KS_SET_P (-1)    /* ks_bconv source set: the P primes (target: Q) */

/* Dataflows of the paper's classification (Qualitative Analysis section). */
#define KS_DSOB 0 /* digits one after another, all output limbs at once */
#define KS_DPOB 1 /* all digits in one launch per stage, all output limbs */
#define KS_DSOC 2 /* digits one after another, output limbs in `chunks` parts */
#define KS_DPOC 3 /* all digits per launch, output limbs in `chunks` parts */
#define KS_STAGED 4 /* ks_modup, ks_keymult and ks_moddown in sequence */

typedef struct ks_params ks_params; /* opaque, immutable after creation */

typedef struct {
  int dataflow; /* KS_DSOB .. KS_STAGED */
  int chunks;   /* output partitions for KS_DSOC / KS_DPOC (1..64), else ignored */
  int log_r;    /* NTT split N = 2^log_r * M: 2^log_r rows per column, blocks of M
                   coefficients (0 = one block pass, up to 5); negative = default */
  int flags;    /* KS_PLAN_MFMA_BCONV | KS_PLAN_SPLIT_STREAMS | KS_PLAN_HOIST_FWD; other bits are rejected (KS_EUNSUP) */
  int batch_tile; /* items per pass: 0 = the whole batch in one pass; else the batch runs in
                     consecutive passes of at most batch_tile items in stream order, each reusing
                     a workspace (and cache footprint) sized for one pass; negative = KS_EUNSUP */
} ks_plan;

/* Plan flag: run ModUp's and ModDown's fast base conversion (the BConv of
   the KeySwitch subsection of the Background section, D_j -> PQ \ D_j and
   P -> Q) as an exact int8 matrix product on the matrix cores: residues and constants are split
   into balanced signed bytes, the int32 partial sums of each byte weight are
   folded back modulo the target prime. The output is identical to the
   default (FP64 / 64-bit integer) BConv. Supported when every digit and P
   have at most 16 primes, log_r <= 5 and the packed digits of a workgroup,
   ceil(max(alpha, k) / 4) * 2^log_r * 2 KB, fit in the 160 KB of LDS
   (ks_keyswitch returns KS_EUNSUP otherwise). */
#define KS_PLAN_MFMA_BCONV 1

/* Plan flag: with batch >= 2, run items [batch/2, batch) on a second stream
   owned by the parameter handle while items [0, batch/2) run on the caller's
   stream, so that the kernels of the two halves share the GPU (one half's
   memory stalls are filled with the other half's arithmetic). The call still
   orders as one unit on the caller's stream: the second stream first waits
   for the work already enqueued there, and the caller's stream waits for the
   second half at the end (also under HIP-graph capture). The workspace is
   the sum of those of the two halves (ks_workspace_bytes). Concurrent calls
   with one handle from several host threads are serialised around this
   fork and join. */
#define KS_PLAN_SPLIT_STREAMS 2

/* Plan flag, with KS_DPOB only (KS_EUNSUP otherwise): run the forward block
   pass of the raised digits as a launch of its own (in place in the
   workspace), then the KeyMult of the P limbs with their inverse block pass,
   and ModDown's last pass with the Q-limb KeyMult, each with one output
   component per workgroup: 6 launches instead of 5, twice the workgroups per
   KeyMult launch and at most one transform per workgroup, for the short
   critical path a single small ciphertext needs (the raised digits make one
   more round trip through memory). The output is identical. */
#define KS_PLAN_HOIST_FWD 4

typedef struct {
  int n, log_n, ell, k, alpha, dnum, ndig;
  int key_ell; /* Q limbs of the evaluation key: ell, or the top level's for a handle of ks_params_at_level */
  uint64_t moduli[KS_MAX_LIMBS]; /* q_0..q_{ell-1}, p_0..p_{k-1} */
  uint64_t psi[KS_MAX_LIMBS];
} ks_info;

/* Derive primes, roots, twiddle tables and BConv constants for (dnum, N =
 * 2^log_n, ell) and upload them to the current HIP device. 3 <= log_n <= 17,
 * 1 <= dnum <= ell, ell + ceil(ell/dnum) <= KS_MAX_LIMBS. The handle is
 * immutable and may be shared by threads and streams of that device.
 * Synchronous (it uploads tables). */
int ks_params_create(int dnum, int log_n, int ell, ks_params** out);
void ks_params_destroy(ks_params* p);

/* The same parameter set at level `level` (1 <= level <= ell of `top`): a
 * ciphertext that has lost its last ell - level limbs, KeySwitched with the
 * top level's evaluation key (the level-aware KeySwitch, which the paper's
 * discussion names as the first way to exploit its per-parameter findings:
 * the work and footprint shrink with the level, so the best plan can change).
 * The level keeps top's P primes, k and alpha; Q becomes q_0..q_{level-1};
 * the digits are top's digits cut at `level` (ndig = ceil(level/alpha)). Every
 * call on the new handle takes and returns data at the level (d [B][level][N],
 * out [B][2][level][N], ext and acc over level + k limbs) but reads the
 * evaluation key in the top level's layout [ndig_top][2][ell_top + k][N]
 * (limb t < level at row t, p_m at row ell_top + m). The new handle is
 * independent of `top` (destroy each with ks_params_destroy). KS_EINVAL for
 * a level outside [1, ell]. ks_bconv on a level handle converts between the
 * level's digits / P and the level's limbs. */
int ks_params_at_level(const ks_params* top, int level, ks_params** out);

/* Host copy of the derived parameters. */
int ks_params_info(const ks_params* p, ks_info* info);

/* Device workspace (bytes) that ks_keyswitch needs for `batch` ciphertexts
 * under `plan` (NULL = default plan); ks_modup and ks_moddown need
 * ks_workspace_bytes(p, batch, &{KS_STAGED}). */
int ks_workspace_bytes(const ks_params* p, int batch, const ks_plan* plan, size_t* bytes);

/* Default plan for these parameters and batch size. */
int ks_default_plan(const ks_params* p, int batch, ks_plan* plan);

/* In-place forward / inverse NTT of x [batch][n_limbs][N]; limb r of each item
 * uses extended-basis prime basis_first + r. The paper names the transform
 * (Background section) but not its root or output order; the order here is
 * the reading stated under "Transform" above (bit-reversed evaluation
 * order, psi the smallest primitive 2N-th root), which every other call
 * assumes for its NTT-form data. KS_EINVAL when the limb range leaves the
 * extended basis. */
int ks_ntt(const ks_params* p, uint64_t* x, int basis_first, int n_limbs, int batch, void* stream);
int ks_intt(const ks_params* p, uint64_t* x, int basis_first, int n_limbs, int batch, void* stream);

/* Fast base conversion in coefficient form. The paper calls the conversion
 * only approximately equivalent to the exact one; this library reads it as
 * the fast conversion without overflow correction (stated under "BConv"
 * above), whose result may exceed the exact one by u*S with
 * 0 <= u < (number of source primes). src_set = digit j: src
 * [batch][|D_j|][N] over D_j -> dst [batch][ell+k-|D_j|][N] over the other limbs
 * of PQ in basis order. src_set = KS_SET_P: src [batch][k][N] over P -> dst
 * [batch][ell][N] over Q. */
int ks_bconv(const ks_params* p, const uint64_t* src, int src_set, uint64_t* dst, int batch, void* stream);

/* ModUp: d [batch][ell][N] (NTT form) -> ext [batch][ndig][ell+k][N] (NTT
 * form); on digit j's own limbs ext holds d unchanged. */
int ks_modup(const ks_params* p, const uint64_t* d, uint64_t* ext, int batch, void* ws, void* stream);

/* KeyMult: acc[b][c][t] = sum_j ext[b][j][t] * evk[j][c][t] mod t for c = 0, 1.
 * evk [ndig][2][ell+k][N] (component 0 = b, 1 = a) is shared by the batch;
 * acc [batch][2][ell+k][N]. */
int ks_keymult(const ks_params* p, const uint64_t* ext, const uint64_t* evk, uint64_t* acc, int batch,
               void* stream);

/* ModDown: acc [batch][2][ell+k][N] -> out [batch][2][ell][N] with
 * out_c = (acc_c,Q - NTT(BConv_{P->Q}(INTT(acc_c,P)))) * P^-1. acc is not modified. */
int ks_moddown(const ks_params* p, const uint64_t* acc, uint64_t* out, int batch, void* ws, void* stream);

/* The whole KeySwitch: d [batch][ell][N] -> out [batch][2][ell][N], with the
 * key evk [ndig][2][ell+k][N]. plan NULL = ks_default_plan. ws must hold
 * ks_workspace_bytes(p, batch, plan) bytes. d, evk and out must not overlap ws. */
int ks_keyswitch(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                 const ks_plan* plan, void* ws, void* stream);

/* ks_keyswitch without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP-graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). The workspace is a
 * static device array of KS_NOALLOC_SCRATCH_BYTES inside the library, one per
 * GPU, held from the first ks_params_create on that GPU until the process
 * ends. The call takes the same arguments as ks_keyswitch minus ws and gives
 * bit-identical output. KS_ETOOBIG (before anything is enqueued) when
 * ks_workspace_bytes(p, batch, plan) exceeds the array: for instance up to
 * 37 items of (2, 2^13, 6) and 5 of (2, 2^15, 10) fit under DPOB, and one of
 * (4, 2^16, 32) under DSOB but not under DPOB. Every call on one GPU uses that GPU's one array: calls that overlap
 * in time on one GPU (several streams, host threads or split plans of
 * different calls) race and give wrong results; the caller orders them. */
#define KS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int ks_keyswitch_noalloc(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                         const ks_plan* plan, void* stream);

/* HMUL (Background section: the product of two ciphertexts followed by
 * relinearisation): for a = (a0, a1) and b = (b0, b1), [batch][2][ell][N]
 * canonical NTT form over the handle's Q (or level),
 *   out = (a0*b0, a0*b1 + a1*b0) + KeySwitch(a1*b1),
 * with evk the key from s*s to s (top-level layout, as ks_keyswitch). The
 * KeySwitch runs under `plan` (NULL = default); a fused plan computes a1*b1
 * in its first pass and adds the other terms in its last, KS_STAGED runs
 * them as kernels of their own. ws: ks_eval_workspace_bytes bytes. out must
 * not alias a or b. Asynchronous on `stream`. */
int ks_hmul(const ks_params* p, const uint64_t* a, const uint64_t* b, const uint64_t* evk, uint64_t* out, int batch,
            const ks_plan* plan, void* ws, void* stream);

/* HROT (Background section: rotation of the slots) by the Galois element
 * `galois` (odd, 0 < galois < 2N; the automorphism x -> x^galois): for
 * ct = (c0, c1) [batch][2][ell][N],
 *   out = (sigma(c0), 0) + KeySwitch(sigma(c1)),
 * with evk the key from sigma(s) to s. This is a reading of the paper's
 * formula, which puts the rotated second component in the first slot and
 * key-switches the rotated first one: with the ciphertext convention of the
 * paper's own HMUL (c0 + c1*s, the second component multiplying the
 * secret), the component to key-switch is the one that multiplies
 * sigma(s), i.e. sigma(c1), and sigma(c0) is kept as it is. In NTT form sigma permutes the slots:
 * slot t of the image is slot t' of the input with
 * 2 brv(t') + 1 = galois * (2 brv(t) + 1) mod 2N. A fused plan gathers
 * sigma(c1) in its first pass and adds sigma(c0) in its last; KS_STAGED runs
 * them as kernels of their own. KS_EINVAL for an even or out-of-range
 * element. out must not alias ct. */
int ks_hrot(const ks_params* p, const uint64_t* ct, int galois, const uint64_t* evk, uint64_t* out, int batch,
            const ks_plan* plan, void* ws, void* stream);

/* Workspace (bytes) of ks_hmul and ks_hrot: the KeySwitch's plus 3*batch*ell*N words. */
int ks_eval_workspace_bytes(const ks_params* p, int batch, const ks_plan* plan, size_t* bytes);

/* Number of kernel launches ks_keyswitch enqueues for (batch, plan). */
int ks_launch_count(const ks_params* p, int batch, const ks_plan* plan);

/* HIP-graph replay of one KeySwitch. ks_graph_create runs
 * ks_keyswitch(p, d, evk, out, batch, plan, ws) once eagerly on `stream` (a
 * non-null hipStream_t), then captures the same call into a HIP graph and
 * instantiates it. Its pointers are baked into the graph: each
 * ks_graph_launch(g, stream) recomputes out from the current contents of d and
 * evk, with one graph launch instead of the plan's kernel launches. The graph
 * holds no memset node. Destroy with ks_graph_destroy; the caller keeps every
 * buffer alive while the graph is in use. Graphs do not record launch traces. */
typedef struct ks_graph ks_graph;
int ks_graph_create(const ks_params* p, const uint64_t* d, const uint64_t* evk, uint64_t* out, int batch,
                    const ks_plan* plan, void* ws, void* stream, ks_graph** graph);
int ks_graph_launch(ks_graph* graph, void* stream);
void ks_graph_destroy(ks_graph* graph);

/* Kernel kinds of the launch trace. */
#define KS_K_INTT_D 0         /* inverse block pass of d (first step of ModUp) */
#define KS_K_MODUP_COLS 1     /* ModUp: inverse column pass, BConv, forward column pass */
#define KS_K_KEYMULT_BLOCKS 2 /* forward block pass of the raised digits + KeyMult (KS_PLAN_HOIST_FWD: KeyMult of
                                 the P limbs and their inverse block pass only) */
#define KS_K_MODDOWN_COLS 3   /* ModDown: inverse column pass, BConv, forward column pass */
#define KS_K_MODDOWN_BLOCKS 4 /* forward block pass + subtraction and P^-1 */
#define KS_K_EXT_BLOCKS 5     /* forward block pass of the raised digits in a launch of its own
                                 (ks_modup, KS_PLAN_HOIST_FWD) */
#define KS_K_PBLOCKS_INV 6    /* ks_moddown: inverse block pass of the P limbs */
#define KS_K_COPY_DIGITS 7    /* ks_modup: digit limbs copied into ext */
#define KS_K_KEYMULT 8        /* ks_keymult element-wise kernel */
#define KS_K_BCONV 9          /* ks_bconv */
#define KS_K_NTT 10           /* ks_ntt / ks_intt passes */
#define KS_K_EVAL 11          /* ks_hmul / ks_hrot element-wise passes */

/* Launch trace (profiling; eager calls only, never under graph capture).
 * After ks_trace_begin, every kernel launch of a kind whose bit is set in
 * kind_mask that this thread enqueues through the library is bracketed by
 * hipEventRecord(events[2i]) and hipEventRecord(events[2i+1]) on its stream,
 * for i = 0 .. capacity-1. `events` holds 2*capacity hipEvent_t created by the
 * caller (as void*). ks_trace_end stops recording, writes the kind of each
 * recorded launch to kinds[0 .. min(n, capacity)-1] and returns n. */
int ks_trace_begin(void** events, int capacity, unsigned kind_mask);
int ks_trace_end(int* kinds, int capacity);

/* Throughput probe of the modular products the kernels are built from (the
 * ALU roofline of the path): blocks x 256 threads each run ks_modmul_chains()
 * independent chains of `iters` dependent products by a fixed residue, for
 * kind 0 the FP64 product modulo the first Q prime (the Q-limb arithmetic),
 * 1 the Shoup product and 2 the Montgomery product modulo the first P prime
 * (the P-limb arithmetic); each thread writes one word of its result to
 * sink [blocks * 256] (a device buffer the caller owns). Time it with events
 * on `stream`: products = blocks * 256 * ks_modmul_chains() * iters.
 * KS_EINVAL for another kind, blocks outside [1, 2^20] or iters < 1. */
int ks_modmul_rate(const ks_params* p, int kind, int blocks, int iters, uint64_t* sink, void* stream);
int ks_modmul_chains(void);

/* HBM copy probe (the practical streaming ceiling of the path): dst[i] =
 * src[i] for `words` 64-bit words, device buffers owned by the caller that
 * must not overlap, blocks x 256 threads in a grid-stride loop, each access
 * 8 bytes (kind 0) or 16 bytes (kind 1, words even), stores non-temporal
 * when nt != 0. Time it with events on `stream`; bytes moved = 16 * words.
 * KS_EINVAL for another kind, an odd count with kind 1, or blocks outside
 * [1, 2^20]. */
int ks_copy_rate(int kind, int nt, int blocks, const uint64_t* src, uint64_t* dst, size_t words, void* stream);

const char* ks_strerror(int code);
/* Name of the HIP error behind the calling thread's last KS_EHIP. */
const char* ks_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
