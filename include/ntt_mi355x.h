/*
 * ntt_mi355x.h -- C ABI of the MI355X (gfx950) exact NTT library.
 *
 * Arithmetic is over F_p for primes p = k 2^l + 1 (section 1 of van der Hoeven,
 * Lecerf, Quintin, "Modular SIMD arithmetic in Mathemagix"): residues are stored
 * canonically in {0, ..., p-1} (section 2) as uint32 when p < 2^31 and uint64 when
 * 2^31 <= p < 2^62.  The transform is the FFT of section 5.1,
 *     a^_i = sum_j w^(i j) a_j,
 * with w = g^((p-1)/n) for the plan's generator g; the bit-reversed ("TFT") order of
 * section 5.1 places a^_[i]_k at position i.
 *
 * Conventions shared by every entry point:
 *  - Every data pointer is a DEVICE pointer (hipMalloc / torch) aligned to its
 *    element size, owned by the caller.  The library owns only plan tables.
 *  - Work is enqueued asynchronously on `hip_stream` (NULL = the default stream).
 *    Argument errors are detected on the host and returned before anything is
 *    enqueued; a failed launch returns NTT_EDEVICE.
 *  - `workspace` is caller-owned device scratch of at least the size reported by
 *    the matching *_workspace_bytes function; it may be NULL when that size is 0.
 *  - Inputs must be canonical residues; only NTT_VALIDATE checks (synchronously).
 *  - No C++ exception crosses this boundary.  Return value: NTT_OK or a negative
 *    error code; ntt_last_error() gives a thread-local detail string.
 */
#ifndef NTT_MI355X_H
#define NTT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NTT_OK = 0,
  NTT_EINVAL = -1,        /* bad argument (NULL pointer, size, alignment, flags) */
  NTT_ENOTPRIME = -2,     /* the modulus is not prime */
  NTT_ENOROOT = -3,       /* 2^log2n does not divide p - 1, or g does not generate F_p^* */
  NTT_ERANGE = -4,        /* NTT_VALIDATE found a non-canonical input */
  NTT_ENOMEM = -5,        /* device allocation of plan tables failed, or workspace too small */
  NTT_EDEVICE = -6,       /* a HIP call or kernel launch failed */
  NTT_EUNSUPPORTED = -7   /* modulus outside [3, 2^62), or size beyond the library's limits */
};

/* Plan flags. */
#define NTT_BITREV_OUT 1u /* forward leaves its output in bit-reversed (TFT) order     */
#define NTT_BITREV_IN 2u  /* inverse takes its input in bit-reversed (TFT) order       */
#define NTT_VALIDATE 4u   /* check that inputs are < p before launching (synchronous)   */
#define NTT_FP64 8u       /* residues held in doubles (section 3, Functions 16-17): vectors of
                             double holding the integers 0 .. p-1, p < 2^50; not with
                             NTT_VALIDATE; transform lengths up to 2^23 */

typedef struct ntt_plan ntt_plan;

typedef struct {
  uint64_t p;         /* modulus                                              */
  uint64_t g;         /* generator of F_p^* used for the roots                */
  uint64_t w;         /* primitive n-th root of unity w = g^((p-1)/n)         */
  uint64_t w_inv;     /* w^-1                                                 */
  uint64_t n_inv;     /* n^-1 mod p                                           */
  uint32_t log2n;     /* transform length n = 2^log2n                        */
  uint32_t word_bits; /* 32 or 64: element type of the plan's vectors         */
  uint32_t flags;     /* NTT_BITREV_OUT | NTT_BITREV_IN | NTT_VALIDATE        */
  uint32_t passes;    /* number of HBM passes of one transform (1 = LDS-resident) */
  uint32_t row_log2;  /* two passes: rows of 2^row_log2 words, columns of n / 2^row_log2 */
} ntt_plan_info;

/* Polynomial-product descriptor for the batched entry point.  a, b, c are device
 * pointers to uint32 (p < 2^31) or uint64 (p >= 2^31) residues; c receives
 * la + lb - 1 coefficients (nothing when la or lb is 0). */
typedef struct {
  uint64_t p;
  const void* a;
  size_t la;
  const void* b;
  size_t lb;
  void* c;
} ntt_polymul_desc;

/* Human-readable name of an error code (static storage). */
const char* ntt_strerror(int code);

/* Detail of the last error returned on the calling thread ("" if none). */
const char* ntt_last_error(void);

/* ---------------------------------------------------------------- host-only helpers
 * These run on the CPU and touch no device. */

/* 1 if n is prime (deterministic Miller-Rabin, valid for every 64-bit n), else 0. */
int ntt_is_prime(uint64_t n);

/* Smallest generator of F_p^* (0 if p is not prime). */
uint64_t ntt_smallest_generator(uint64_t p);

/* Largest prime p < 2^bits with p = 1 mod 2^l (p = k 2^l + 1), 0 if none;
 * bits <= 63.  ntt_find_prime(62, 32) is the serving mix's ~62-bit prime. */
uint64_t ntt_find_prime(uint32_t bits, uint32_t l);

/* ---------------------------------------------------------------- transforms
 * Section 5.1: FFT_w of length n = 2^log2n over F_p. */

/* Create a plan for length 2^log2n (0 <= log2n <= l where p = k 2^l + 1) modulo p.
 * g = 0 selects the smallest generator; otherwise g must generate F_p^*.
 * The plan precomputes and uploads its twiddle tables (section 5.1 caches every
 * root and power the transforms need) with synchronous copies; `hip_stream` is unused at creation and may be NULL.
 * A plan is immutable after creation and may be used concurrently on different
 * streams.  Errors: NTT_EINVAL (out == NULL, unknown flags), NTT_EUNSUPPORTED
 * (p < 3 or p >= 2^62, log2n > 26), NTT_ENOTPRIME, NTT_ENOROOT, NTT_ENOMEM. */
int ntt_plan_create(ntt_plan** out, uint64_t p, uint64_t g, uint32_t log2n, uint32_t flags, void* hip_stream);

/* Free a plan and its device tables.  NULL is accepted.  The caller must make sure
 * no enqueued work still uses it. */
int ntt_plan_destroy(ntt_plan* plan);

int ntt_plan_get_info(const ntt_plan* plan, ntt_plan_info* info);

/* Device scratch needed by ntt_forward / ntt_inverse for `batch` vectors. */
size_t ntt_workspace_bytes(const ntt_plan* plan, size_t batch);

/* Forward transform of `batch` vectors of n residues.  Vector b starts at
 * in + b * stride_elems (elements, stride_elems >= n).  in == out is allowed.
 * Output order: natural (out_i = a^_i), or bit-reversed with NTT_BITREV_OUT.
 * Errors: NTT_EINVAL (NULL/misaligned pointer, stride < n), NTT_ENOMEM (workspace
 * too small), NTT_ERANGE (NTT_VALIDATE only), NTT_EDEVICE. */
int ntt_forward(const ntt_plan* plan, const void* in, void* out, size_t batch, size_t stride_elems,
                void* workspace, size_t ws_bytes, void* hip_stream);

/* Inverse transform: FFT_{w^-1} followed by multiplication by n^-1, so that
 * ntt_inverse(ntt_forward(a)) = a exactly (section 5.1: invert the steps and use the
 * inverse transform).  Input order natural, or bit-reversed with NTT_BITREV_IN.
 * Same arguments and errors as ntt_forward. */
int ntt_inverse(const ntt_plan* plan, const void* in, void* out, size_t batch, size_t stride_elems,
                void* workspace, size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------- truncated transforms
 * Section 5.1: the truncated Fourier transform of an l-tuple (a_0, ..., a_(l-1)) is
 *     TFT(a) = (A(w^[0]_k), ..., A(w^[l-1]_k)),  A(X) = a_0 + a_1 X + ... + a_(l-1) X^(l-1),
 * the first l values of the transform in the TFT (bit-reversed) order, n = 2^k the
 * plan's length.  Algorithm 1 computes it with n1 = 2^row_log2 (ntt_plan_get_info):
 * only the first ceil(l / n1) rows of its step 3 run; one-pass plans transform whole
 * vectors in LDS.  The inverse recovers the l coefficients from the l values by the
 * inverse TFT (invert steps 4 to 1 of Algorithm 1 with the inverse TFT on the columns,
 * and on the one row that a general l leaves partially known).
 * Supported: plans of 32- or 64-bit words whose columns are at most 2^10 words (n <=
 * 2^24 for the default row lengths); others return NTT_EUNSUPPORTED.  The plan's flags
 * (bit orders) do not apply: input coefficients are in natural order, values in TFT order. */

/* Device scratch of ntt_tft_forward / ntt_tft_inverse for `batch` vectors (0 for
 * one-pass plans). */
size_t ntt_tft_workspace_bytes(const ntt_plan* plan, size_t batch);

/* out[b * out_stride + i] = A_b(w^[i]_k) for i < l_out, where A_b has the l_in
 * coefficients in[b * in_stride + j], j < l_in (zero above), for b < batch.
 * 0 <= l_in, l_out <= n, l_in <= in_stride, l_out <= out_stride.
 * Errors: NTT_EINVAL (NULL/misaligned pointers, lengths), NTT_ENOMEM (workspace),
 * NTT_EUNSUPPORTED (plan shape, residues in doubles), NTT_EDEVICE. */
int ntt_tft_forward(const ntt_plan* plan, const void* in, size_t l_in, void* out, size_t l_out, size_t batch,
                    size_t in_stride, size_t out_stride, void* workspace, size_t ws_bytes, void* hip_stream);

/* The inverse: out[b * out_stride + j], j < l, receives the unique coefficients whose
 * first l TFT values are in[b * in_stride + i], i < l (canonical residues).  0 <= l <= n.
 * Errors as ntt_tft_forward. */
int ntt_tft_inverse(const ntt_plan* plan, const void* in, void* out, size_t l, size_t batch, size_t in_stride,
                    size_t out_stride, void* workspace, size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------- polynomial products
 * Section 5.2: the product of two polynomials over F_p by two forward transforms,
 * an entry-wise product and one inverse transform, after zero padding to the
 * transform length N = the smallest power of two >= la + lb - 1. */

size_t polymul_workspace_bytes(uint64_t p, size_t la, size_t lb);

/* c[0 .. la+lb-2] = a * b mod p (linear product; c has la + lb - 1 entries).
 * la == 0 or lb == 0: nothing is written, NTT_OK.  Element type: uint32 when
 * p < 2^31, else uint64.  Plans (tables) are created on first use per (device, p)
 * and cached for the life of the process.
 * Errors: NTT_EINVAL, NTT_ENOTPRIME, NTT_ENOROOT (N > 2^l), NTT_EUNSUPPORTED,
 * NTT_ENOMEM, NTT_EDEVICE. */
int polymul_modp(uint64_t p, const void* a, size_t la, const void* b, size_t lb, void* c, void* workspace,
                 size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same product as polymul_modp,
 * with the same arguments minus the workspace, which is instead a fixed array of
 * NTT_NOALLOC_SCRATCH_BYTES in device memory that the library holds on every device
 * it runs on until the process ends.  The call allocates nothing (no hipMalloc, no
 * host staging) and so creates no plan: the plan of (p, N) must already be cached on
 * the current device, which any earlier polymul_modp call with the same modulus and
 * transform length does.  Nothing in the array needs to start at zero; every call
 * writes what it reads.  All calls on one device share its array: calls whose work
 * can overlap on the device (different streams, or host threads racing on one) race
 * on it and give wrong results; serialize them on one stream.
 * Errors: as polymul_modp, plus NTT_EINVAL when the plan is not cached yet and
 * NTT_ENOMEM when the product needs more scratch than the array holds (two-pass
 * products: 2 N words, i.e. N <= 2^22 for 32-bit words and N <= 2^21 for 64-bit). */
#define NTT_NOALLOC_SCRATCH_BYTES (32u << 20)
int polymul_modp_noalloc(uint64_t p, const void* a, size_t la, const void* b, size_t lb, void* c, void* hip_stream);

/* Device scratch for polymul_modp_batch on these descriptors. */
size_t polymul_batch_workspace_bytes(const ntt_polymul_desc* d, size_t count);

/* All `count` products in as few launches as the sizes allow: the descriptors
 * whose transform fits one workgroup (N <= 2^16 for 32-bit, 2^15 for 64-bit
 * primes) are grouped by word size and size class (the classes differ in
 * workgroup size and LDS), and each group is ONE persistent fused launch (fold,
 * forward x2, entry-wise product, inverse, combine) whatever the primes and
 * lengths of its products (section 2.2, Remark 6: several moduli in one vector
 * launch); the larger products run the multi-pass path one after another.  The
 * groups' launches and the multi-pass sequence are independent: the first runs on
 * hip_stream, the others on streams forked from it (an event) and joined back into it
 * before the call returns, so that they overlap on the device; hip_stream orders
 * everything the call enqueues, as if it had run there alone (while a graph is being
 * captured, or with the tuning choice "batch.fork" = 0, everything runs on hip_stream).
 * `d` is a HOST array; its content is copied into the workspace.
 * Errors as polymul_modp, checked for every descriptor before anything runs. */
int polymul_modp_batch(const ntt_polymul_desc* d, size_t count, void* workspace, size_t ws_bytes,
                       void* hip_stream);

/* Reusable batch: the descriptors are checked, their plans created and their
 * device form uploaded once (synchronously) into device memory the handle owns;
 * every launch then only enqueues kernels on `hip_stream` and on the streams its
 * launches fork onto, joined back into `hip_stream` as in polymul_modp_batch (nothing
 * is copied or allocated on the device; the first launch from a stream creates the
 * streams it forks onto), so a launch can be repeated, overlapped on several streams
 * when the operands differ, or captured in a HIP graph (captured launches stay on
 * `hip_stream`).  The operand pointers are bound at creation.  Errors as
 * polymul_modp_batch. */
typedef struct ntt_batch ntt_batch;
int polymul_batch_create(ntt_batch** out, const ntt_polymul_desc* d, size_t count);
/* Device scratch needed by polymul_batch_launch: a park area for each launch of
 * 2^14..2^16-point products (32-bit primes) and the largest multi-pass product's
 * scratch; 0 when there is neither. */
size_t polymul_batch_launch_workspace_bytes(const ntt_batch* batch);
int polymul_batch_launch(const ntt_batch* batch, void* workspace, size_t ws_bytes, void* hip_stream);
/* NULL is accepted; the caller makes sure no launch of the batch is still pending. */
int polymul_batch_destroy(ntt_batch* batch);

/* ---------------------------------------------------------------- tuning
 * Launch-shape choices the kernels support, picked per size by the autotuner that
 * ships with the Python package (it times every candidate on the device, checks
 * that all candidates give identical results and writes a text file of choices).
 * Keys and values:
 *   "split.w32.L<L>"  (15 <= L <= 26) row length log2 of two-pass transform plans
 *                     created by ntt_plan_create: 12, 13 or 14 (default 14)
 *   "split.w64.L<L>"  (14 <= L <= 26) the same for 64-bit primes: 12 or 13 (default 13)
 *   "psplit.w32.L<L>", "psplit.w64.L<L>"  the same for the plans the products cache
 *   "fused.single.max.w32"  largest log2 N at which a single product (polymul_modp,
 *                     each prime of intmul_crt) takes the fused one-workgroup kernel:
 *                     14, 15 or 16 (default 16); above it the two-pass path (batches
 *                     keep the fused kernel up to 2^16)
 *   "fused.single.max.w64"  the same for 64-bit primes: 13, 14 or 15 (default 15)
 *   "batch.fork"     1 (default): a batch's size classes and multi-pass products run on
 *                     forked streams (polymul_modp_batch, polymul_batch_launch); 0: all on
 *                     the caller's stream
 *   "fused.m15.w32"  1: fused products of transform length 2^16 over 32-bit primes
 *                     run as two sub-problems of 2^15 points (one operand's
 *                     transform held in registers); 0 (default): four of 2^14
 *   "single.split.w32.L<L>" (11 <= L <= 16), "single.split.w64.L<L>" (11 <= L <= 15)
 *                     a single product of length 2^L runs its 2^d sub-problems of
 *                     2^(L-d) points on 2^d workgroups at once, then recombines them
 *                     (latency path; workspace N words): d = 1, 2 or 3 with
 *                     10 <= L - d <= 13 (32-bit) / 12 (64-bit), or 0 (default: off)
 *   "server.copy_threads"  host threads that copy operands into and products out of a
 *                     serving loop's staging: 0 .. 63 (default 7; 0: the driving thread
 *                     copies), read by ntt_server_create
 *   "server.batches_per_stream"  batches a serving loop keeps in flight per stream, each
 *                     with its own staging block: 1 .. 8 (default 2), read by
 *                     ntt_server_create
 *   "tft.rows.w32", "tft.rows.w64"  1: two-pass products run only the first
 *                     ceil(lc / 2^row_log2) rows of their transforms (section 5.1's TFT)
 *                     and invert the columns by the inverse TFT; 0 (default): full-length
 *                     transforms
 * A choice applies to plans created afterwards: clear the plan cache to re-plan.
 * Every choice computes the same (unique, canonical) results.
 * ntt_tune_set / ntt_tune_get: NTT_EINVAL for an unknown key, a value out of range
 * or (get) a key that is not set.  ntt_tune_load reads "key value" lines ('#'
 * starts a comment) and applies all of them or, on any bad line, none (NTT_EINVAL).
 * ntt_plan_cache_clear destroys the cached plans of the current device (waits for
 * the device); batch handles and graphs made before it must not be used again. */
int ntt_tune_set(const char* key, int64_t value);
int ntt_tune_get(const char* key, int64_t* value);
int ntt_tune_clear(void);
int ntt_tune_load(const char* path);
int ntt_plan_cache_clear(void);

/* ---------------------------------------------------------------- HIP graphs
 * Launch-bound callers (many small products, a serving loop) replay a recorded
 * sequence of library calls as one graph launch instead of issuing every kernel.
 * ntt_graph_begin starts recording `hip_stream` (a created stream, not the null
 * stream; thread-local capture mode); every library call made on that stream by
 * this thread until ntt_graph_end is recorded, not run.  ntt_graph_end closes the
 * recording and instantiates it.  A replay (ntt_graph_launch) reruns the recorded
 * kernels on the same device pointers, reading whatever the buffers hold then.
 * Recordable: polymul_batch_launch, intmul_crt, polymul_modp, ntt_forward and
 * ntt_inverse without NTT_VALIDATE, once the plans they use exist (run each call
 * once before recording it).  Refused with NTT_EINVAL while recording (nothing is
 * enqueued, the recording stays usable): calls that would create a plan, allocate,
 * copy host data (polymul_modp_batch) or wait (NTT_VALIDATE).  Recorded graphs hold
 * no memset nodes.  The caller owns the graph and destroys it once no replay is
 * pending.  Errors: NTT_EINVAL, NTT_EDEVICE (the HIP capture or instantiation
 * failed, e.g. because another call on the stream was not recordable). */
typedef struct ntt_graph ntt_graph;
int ntt_graph_begin(void* hip_stream);
int ntt_graph_end(void* hip_stream, ntt_graph** out);
int ntt_graph_launch(const ntt_graph* graph, void* hip_stream);
int ntt_graph_destroy(ntt_graph* graph);

/* ---------------------------------------------------------------- integer product
 * Section 5.3: Kronecker segmentation with 16-bit chunks (A(2^16) = a) and the
 * three-prime transform over p1 = 998244353, p2 = 469762049, p3 = 167772161,
 * Chinese remaindering (Garner) and carry propagation. */

size_t intmul_workspace_bytes(size_t na, size_t nb);

/* c = a * b for nonnegative integers given as little-endian 16-bit limbs (device
 * pointers).  c receives exactly ceil((na + nb) / 2) little-endian 32-bit limbs,
 * unnormalised (leading zero limbs allowed).  na == 0 or nb == 0 writes zeros.
 * Errors: NTT_EINVAL (NULL pointers, na + nb - 1 > 2^23: the smallest 2-adic
 * order of the three primes is 23), NTT_ENOMEM (workspace), NTT_EDEVICE. */
int intmul_crt(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint32_t* c, void* workspace,
               size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------- serving
 * A request loop on the current device: requests (polynomial products mod p with
 * host residue vectors, kind 0; integer products of host 16-bit limbs, kind 1) are
 * queued by ntt_server_submit and served by ntt_server_progress, which (1) completes
 * the batches whose work has finished, copying each product into the request's host
 * buffer c (la + lb - 1 residues, or ceil((la + lb) / 2) 32-bit limbs) and reporting
 * the request ids, and (2) admits pending requests in arrival order while the HBM
 * budget has room: consecutive polynomial requests form one polymul_modp_batch call,
 * an integer product one intmul_crt call, each batch with one upload and one download
 * through page-locked staging, on one of `streams` streams (default priority).
 * Batches in flight overlap on the device (at most 2 per stream by default).  The
 * host copies into and out of staging run on the server's copy threads while the
 * device works; ntt_server_progress itself never waits for them.  c == NULL: the
 * product is computed but not copied back; c in page-locked host memory (hipHostMalloc,
 * torch pin_memory): the product is copied there directly by DMA, without staging.  The server owns one device buffer of
 * hbm_budget bytes (the arena) and its page-locked staging (32 MiB per batch in
 * flight, allocated at creation); the caller keeps a, b and c valid until the
 * request's id is reported.  One host thread drives a server.
 * Errors: NTT_EINVAL (arguments), NTT_ENOTPRIME / NTT_ENOROOT (kind 0 prime or length),
 * NTT_ENOMEM (a request that cannot fit the budget even alone; allocation failures),
 * NTT_EDEVICE (a device failure: destroy the server). */
typedef struct ntt_server ntt_server;
int ntt_server_create(ntt_server** out, size_t hbm_budget, int streams, size_t max_batch);
int ntt_server_submit(ntt_server* server, uint64_t id, int kind, uint64_t p, const void* a, size_t la,
                      const void* b, size_t lb, void* c);
/* done_ids receives at most cap ids of completed requests, *ndone how many; completed
 * requests beyond cap are handed back by later calls (stats count them as in flight).
 * If a batch cannot be enqueued (NTT_EDEVICE, NTT_ENOMEM), its requests return to the
 * front of the queue and its memory to the arena before the error is returned. */
int ntt_server_progress(ntt_server* server, uint64_t* done_ids, size_t cap, size_t* ndone);
int ntt_server_stats(const ntt_server* server, size_t* pending, size_t* inflight, size_t* arena_used,
                     size_t* max_inflight);
/* Waits for the work in flight, then frees everything the server owns. */
int ntt_server_destroy(ntt_server* server);

/* Section 5.3's choice of the chunk size h for integers of na16 and nb16 16-bit
 * limbs: the largest h in {32, 16} with 2^(2h + ceil(log2(d + 1))) < p1 p2 p3 (d the
 * larger chunk count) and d_a + d_b - 1 <= 2^23; 0 when neither fits. */
int intmul_chunk_bits(size_t na16, size_t nb16);

size_t intmul32_workspace_bytes(size_t na, size_t nb);

/* c = a * b for nonnegative integers given as little-endian 32-bit chunks (h = 32:
 * half the transform length of the 16-bit path for the same integers; a 16-bit-limb
 * integer with an even limb count is the same array read as 32-bit chunks).  c
 * receives exactly na + nb little-endian 32-bit limbs, unnormalised.  Each chunk is
 * reduced modulo each prime first (2^32 exceeds them).  na == 0 or nb == 0 writes
 * zeros.  Errors: NTT_EINVAL (NULL or misaligned pointers; min(na, nb) (2^32 - 1)^2
 * reaching p1 p2 p3, about min(na, nb) > 4.26e6; na + nb - 1 > 2^23), NTT_ENOMEM
 * (workspace), NTT_EDEVICE. */
int intmul_crt32(const uint32_t* a, size_t na, const uint32_t* b, size_t nb, uint32_t* c, void* workspace,
                 size_t ws_bytes, void* hip_stream);

/* Polynomial matrix product (section 5.2): C = A B for n x n matrices over F_p[x]
 * whose entries have degree < d, through transforms of length N = 2^ceil(log2(2d - 1))
 * of every entry, one n x n matrix product over F_p per frequency, and the inverse
 * transforms of C's entries.
 * A, B: device, n*n*d canonical residues (uint32) each; entry (i, j) holds its d
 *   coefficients, lowest degree first, at offset (i*n + j)*d.
 * C: device, n*n*(2d - 1) canonical residues; entry (i, j) at (i*n + j)*(2d - 1).
 * p: prime below 2^31 with 2^ceil(log2(2d - 1)) dividing p - 1.  1 <= n <= 64.
 * workspace: device, polymatmul_workspace_bytes(p, n, d) bytes (2 n^2 N words),
 *   256-byte aligned, owned by the caller.  Asynchronous on hip_stream.
 * n == 0 or d == 0: nothing to do, NTT_OK.
 * Errors: NTT_ENOTPRIME, NTT_ENOROOT, NTT_EUNSUPPORTED (p >= 2^31, n > 64),
 *   NTT_EINVAL (NULL or misaligned pointers, d > 2^25), NTT_ENOMEM (workspace too small),
 *   NTT_EDEVICE (launch failure). */
size_t polymatmul_workspace_bytes(uint64_t p, size_t n, size_t d);
int polymatmul_modp(uint64_t p, size_t n, const void* A, const void* B, size_t d, void* C, void* workspace,
                    size_t ws_bytes, void* hip_stream);

/* Integer matrix product (section 5.3): C = A B for n x n matrices of nonnegative
 * integers, through Kronecker segmentation into chunks of 32 bits (section 5.3's
 * chunk size for these primes), the polynomial matrix product modulo each of
 * 998244353, 469762049 and 167772161 (polymatmul_modp), and per entry Garner's
 * reconstruction and the carries.
 * A, B: device, n*n entries of na little-endian 32-bit limbs each, entry (i, j) at
 *   offset (i*n + j)*na.  C: device, n*n entries of 2*na + 1 limbs, entry (i, j) at
 *   (i*n + j)*(2*na + 1), unnormalised (leading zero limbs).
 * 1 <= n <= 64; n * na * (2^32 - 1)^2 < p1 p2 p3 (about 2^86; n = 32 allows na up to
 *   2^16) and 2*na - 1 <= 2^23.  workspace: intmatmul32_workspace_bytes(n, na) bytes.
 * n == 0 or na == 0: nothing to do, NTT_OK.
 * Errors: NTT_EINVAL (pointers, sizes beyond the bounds), NTT_EUNSUPPORTED (n > 64),
 *   NTT_ENOMEM (workspace), NTT_EDEVICE. */
size_t intmatmul32_workspace_bytes(size_t n, size_t na);
int intmatmul_crt32(size_t n, const uint32_t* A, const uint32_t* B, size_t na, uint32_t* C, void* workspace,
                    size_t ws_bytes, void* hip_stream);

/* Element-wise evaluation of one device primitive on n elements (a diagnostic for
 * testing the arithmetic alone; every transform kernel uses these same forms).
 * word: 32 or 64 (unsigned words, p < 2^31 or p < 2^62) or 0 (doubles, p < 2^50).
 * x, y, ys, out: device arrays of the word type (ys: Shoup companions
 * floor(y 2^W / p), op NTT_ARITH_SHOUP with unsigned words only; out: n words, 2n for
 * the butterflies).  tw, tws: the butterflies' twiddle and its companion (the same in
 * every lane); for doubles only tw is read.  Lazy ranges as in the kernels: unsigned
 * 32-bit words lazy when p < 2^30, 64-bit words always, doubles when p < 2^48.
 * Errors: NTT_EINVAL (op, word, p even or < 3, NULL or misaligned pointers),
 * NTT_EUNSUPPORTED (p beyond the word's bound), NTT_EDEVICE. */
#define NTT_ARITH_SHOUP 0 /* out = x y - floor(x ys / 2^W) p, in [0, 2p) for any word x (Function 8
                             without its last line); doubles: Function 16, [0, 2p) */
#define NTT_ARITH_MONT 1  /* out = x y 2^-W mod p, in (0, 2p), for x y < 2^W p (Function 13,
                             subtractive form); doubles: Function 16, x y mod p in [0, 2p) */
#define NTT_ARITH_RED1 2  /* out = x - p if x >= p else x (Function 2's min): [0, 2p) -> [0, p) */
#define NTT_ARITH_RED2 3  /* out = x - 2p if x >= 2p else x: [0, 4p) -> [0, 2p) */
#define NTT_ARITH_CT 4    /* forward butterfly: out[i] = X + w Y, out[n + i] = X - w Y mod p,
                             lazy: X in [0, 4p) -> [0, 4p); else X in [0, 2p) -> [0, 2p) */
#define NTT_ARITH_GS 5    /* inverse butterfly: out[i] = X + Y, out[n + i] = (X - Y) w mod p,
                             lazy: [0, 2p) -> [0, 2p); else [0, p) -> [0, p) */
int ntt_arith_apply(int op, int word, uint64_t p, const void* x, const void* y, const void* ys, uint64_t tw,
                    uint64_t tws, void* out, size_t n, void* hip_stream);

/* Products mod p with residues held in doubles (section 3: modular arithmetic over
 * numeric types; products by Function 16, the FMA product, sums by Function 17's
 * compare-and-subtract), in the same fused one-workgroup kernels as polymul_modp_batch
 * for transforms up to 2^15 and in the two-pass kernels above.
 * Descriptors as for polymul_modp_batch, except that a, b and c point to device arrays
 * of double holding canonical residues (integers in [0, p)); c receives la + lb - 1
 * canonical residues as doubles.
 * p: prime below 2^50 (Function 16 needs x y < 2^50 p: operands stay below 4p between
 *   butterflies for p < 2^48, and multiplicands are reduced to [0, p) first above);
 *   transform length 2^ceil(log2(la + lb - 1)) at most 2^23 and dividing p - 1.
 * workspace: polymul_f64_batch_workspace_bytes(d, count) bytes (the device copy of the
 *   descriptors and the two-pass products' transforms).  Asynchronous on hip_stream;
 *   not recordable in a graph.
 * Errors: NTT_EUNSUPPORTED (p >= 2^50, transform longer than 2^23), NTT_ENOTPRIME,
 *   NTT_ENOROOT, NTT_EINVAL (NULL or misaligned pointers, graph capture), NTT_ENOMEM
 *   (workspace too small), NTT_EDEVICE. */
size_t polymul_f64_batch_workspace_bytes(const ntt_polymul_desc* d, size_t count);
int polymul_f64_batch(const ntt_polymul_desc* d, size_t count, void* workspace, size_t ws_bytes, void* hip_stream);
/* The same products as a reusable batch handle (checked, planned and uploaded once):
 * run with polymul_batch_launch (workspace polymul_batch_launch_workspace_bytes),
 * freed with polymul_batch_destroy; launches are recordable in a graph.  Errors as
 * polymul_f64_batch. */
int polymul_f64_batch_create(ntt_batch** out, const ntt_polymul_desc* d, size_t count);

#ifdef __cplusplus
}
#endif

#endif /* NTT_MI355X_H */
