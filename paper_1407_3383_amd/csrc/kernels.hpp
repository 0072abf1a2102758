// Kernel launch interface used by the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "ntt_lds.hpp"

namespace nttgpu {

// Word code of residues held in doubles (section 3's numeric types) in the launchers'
// word_bits argument; 32 and 64 are the integer words.
constexpr int kWordF64 = -64;

struct FusedBatch {
  const FusedItem* items;  // device array, or NULL to use `single`
  void* park;              // workspace for parked partial results (fused_park_words per workgroup)
  int count;
  int pad;
  FusedItem single;
};

int fused_class(int word_bits, int log2n);
constexpr int kFusedClasses = 5;  // class 4: 32-bit transforms of 2^16 as two 2^15-point sub-problems
int fused_max_log2n(int word_bits);
size_t fused_park_words(int word_bits, int cls);
int fused_grid(int word_bits, int cls, size_t count, int cus);
hipError_t launch_fused(int word_bits, int cls, const FusedBatch& batch, int grid, hipStream_t stream);
// Residues held in doubles, p < 2^49 (classes and grids of the 64-bit word size).
hipError_t launch_fused_f64(int cls, bool band, const FusedBatch& batch, int grid, hipStream_t stream);

// Transform of `batch` vectors that fit one workgroup's LDS (log2n <= lds_max_log2n).
struct LdsNttArgs {
  const void* in;
  void* out;
  uint64_t stride;  // elements between vectors
  const void* pc;   // PassConst<T>
  const void* tw;   // universal tables
  const void* twi;
  uint32_t L;
  uint32_t bitrev;  // forward: leave TFT order; inverse: input in TFT order
  uint32_t batch;
  uint32_t nin;     // forward: input elements per vector (the rest read as 0); 0 = all
  uint32_t nout;    // forward: output elements stored per vector; 0 = all
  uint32_t pad;
  uint64_t out_stride;  // elements between output vectors; 0 = stride
};
int lds_max_log2n(int word_bits);
hipError_t launch_lds_ntt(int word_bits, bool inverse, const LdsNttArgs& a, hipStream_t stream);

// Two-pass transform (section 5.1, Algorithm 1 with n1 = 2^L1 columns of the
// row-major 2^L1 x 2^L2 layout and rows of length 2^L2).
struct PassArgs {
  const void* in;   // pass input (column forward pass: may be uint16_t limbs)
  void* out;        // pass output
  const void* in2;  // second operand (fused product row pass)
  uint64_t in_stride, out_stride;  // elements between batch vectors
  uint64_t valid;   // column forward pass: input elements at index >= valid read as 0
  const void* pc;   // PassConst<T>
  const void* tw;   // universal tables (stages of the column pass / the row transform)
  const void* twi;
  const void* tlo;  // two-level twist tables (forward, inverse, inverse * n^-1)
  const void* thi;
  const void* tilo;
  const void* tihi;
  uint32_t batch;
  uint32_t scale;   // column forward pass: 1 multiply inputs by sigma (second operand of a product),
                    // 2 reduce inputs modulo p (words that may exceed p), 0 neither
  uint32_t in_u16;  // column forward pass: input is 16-bit limbs
  uint32_t rows;    // rows of each vector that are needed (truncated transforms: the first
                    // `rows` rows of the TFT order); 0 = all 2^L1.  Column forward pass:
                    // only these rows are stored; row passes: only these rows run.
};
// Up to kMaxPassJobs passes of the same shape (word, L1, L2, batch, input type) whose
// workgroups share one launch: job = blockIdx.y (several primes, both operands).
constexpr int kMaxPassJobs = 6;
struct PassJobs {
  PassArgs j[kMaxPassJobs];
  int n;
};
hipError_t launch_col_fwd_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_col_inv_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_row_polymul_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_row_fwd_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_col_fwd(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_col_inv(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_row_fwd(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_row_inv(int word_bits, const PassArgs& a, int L1, int L2, bool scale_ninv, hipStream_t stream);
hipError_t launch_row_polymul(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
int pass_max_row_log2(int word_bits);
int pass_col_tile_log2(int word_bits);

// Inverse truncated transforms (section 5.1: Algorithm 1 inverted, steps 4 to 1, with
// the inverse TFT).  Vectors of 2^L = 2^L1 rows x 2^L2 columns (two-pass plans) or one
// LDS-resident vector (2^L <= 2^14 for 32-bit words, 2^13 for 64-bit).
struct TftArgs {
  const void* in;       // TFT values (row-major in the TFT order) or column-domain values
  void* out;
  uint64_t in_stride, out_stride;
  uint64_t valid;       // outputs stored per vector: positions < valid
  const void* pc;       // PassConst<T>
  const void* tw;       // universal tables
  const void* twi;
  const void* tlo;      // two-level twist tables: forward, inverse (without n^-1)
  const void* thi;
  const void* tilo;
  const void* tihi;
  void* rowbuf;         // two-pass general inverse: the twisted column values of the last
                        // row at columns >= lastn (rowbuf_stride words per vector)
  uint64_t rowbuf_stride;
  uint64_t zeta;        // column pass with `eval_next`: w_(2^L1)^([lam]_L1) and its companion
  uint64_t zeta_s;
  double zeta_d;        // the same as a double (residues held in doubles)
  uint32_t lam;         // known TFT values (rows for columns, elements for one vector)
  uint32_t c_lo, c_hi;  // columns processed: [c_lo, c_hi)
  uint32_t eval_next;   // column pass: also evaluate each column's TFT at position lam and
                        // write it, twisted by w_N^([lam]_L1 c), to rowbuf
  uint32_t lastrow;     // row pass: the row index r (= lam - 1 of the columns)
  uint32_t L, L1, L2;
  uint32_t batch;
};
// Column inverse TFT: each column of 2^L1 words holds `lam` known values (rows < lam of
// `in`) and zero inputs below; the first lam inputs are recovered and stored.
hipError_t launch_col_itft(int word_bits, const TftArgs& a, hipStream_t stream);
// One row (r = lastrow) of 2^L2 words per vector: `lam` TFT values from `in` (positions
// r 2^L2 + c, c < lam), known twisted column values at c >= lam from rowbuf; the
// untwisted values at c < lam are written to out (row r).
hipError_t launch_row_itft(int word_bits, const TftArgs& a, hipStream_t stream);
// One LDS-resident vector of 2^L words per batch item: lam TFT values, zero inputs
// above; the lam inputs are stored.
hipError_t launch_vec_itft(int word_bits, const TftArgs& a, hipStream_t stream);

// out[i] = in[[i]_L] for `batch` vectors of 2^L elements (bit-reversal permutation).
hipError_t launch_bitrev_permute(int word_bits, const void* in, void* out, uint64_t in_stride, uint64_t out_stride,
                                 uint32_t L, uint32_t batch, hipStream_t stream);

// x[0 .. n) = value.
hipError_t launch_fill_u32(uint32_t* x, uint64_t n, uint32_t value, hipStream_t stream);

// u16 limbs -> u32 residues (every prime of the integer product exceeds 2^16).
hipError_t launch_widen_u16(const uint16_t* in, uint32_t* out, uint64_t n, hipStream_t stream);

// Element-wise checks for NTT_VALIDATE: sets *flag to 1 if any element >= p.
hipError_t launch_range_check(int word_bits, const void* x, uint64_t n, uint64_t stride, uint32_t batch, uint64_t p,
                              uint32_t* flag, hipStream_t stream);

// Integer product: Garner reconstruction + carry propagation into 32-bit limbs.
// Raises a kernel's dynamic-LDS limit to `bytes` the first time a launch needs it
// (the attribute is process-wide), so repeated and graph-captured launches make no
// attribute call.
hipError_t allow_dynamic_lds(const void* kernel, size_t bytes);

// One product on 2^d workgroups (latency path); park holds the 2^d partials (N words).
struct SplitArgs {
  const void* a;
  const void* b;
  void* c;
  uint64_t la, lb;
  const void* cst;  // PolyConst<T> of the plan
  const void* tw;
  const void* twi;
  void* park;
  uint32_t lam;  // sub-problems computed: ceil(lc / S) (TFT truncation), the rest completed
  uint32_t pad;
};
bool split_supported(int word_bits, int log2n, int d);
hipError_t launch_split(int word_bits, const SplitArgs& a, int log2n, int d, hipStream_t stream);

struct CrtArgs {
  const uint32_t* r1;
  const uint32_t* r2;
  const uint32_t* r3;
  uint64_t lc;       // number of coefficients (na + nb - 1)
  uint64_t npos;     // number of 16-bit output positions (na + nb), even-padded
  uint32_t* t;       // workspace: column sums with one level of carry applied, whole blocks
  uint32_t* blk;     // workspace: per-block (generate, propagate) then carry-in
  uint32_t* c;       // output: npos / 2 limbs of 32 bits
  uint32_t p1, p2, p3;
  uint32_t c12, c12s;    // p1^-1 mod p2 and its Shoup companion
  uint32_t c123, c123s;  // (p1 p2)^-1 mod p3 and companion
  uint32_t p1m3, p1m3s;  // p1 mod p3 and companion
  uint64_t p1p2;
  // batches of independent integers (32-bit chunk tail only): entry e = blockIdx.y
  // reads r_k + e rstride, uses t + e tstride and blk + e bstride, writes c + e cstride
  uint64_t rstride, tstride, cstride;
  uint32_t bstride, batch;  // batch 0 or 1: one integer
};
int crt_block_positions();
hipError_t launch_crt_carry(const CrtArgs& a, hipStream_t stream);
// 32-bit chunks: t holds whole blocks of 64-bit column sums, c gets npos 32-bit limbs.
hipError_t launch_crt32_carry(const CrtArgs& a, hipStream_t stream);
hipError_t launch_reduce_mod(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t p, hipStream_t stream);

// Polynomial matrix product, entry-wise step: C[e][k] for every frequency k < N of the
// n x n matrices whose entries e = i n + j are vectors of N words (A, B: transforms,
// canonical).  C = (sum_l A[i n + l][k] B[l n + j][k]) 2^-32 K mod p, canonical.
constexpr uint32_t kMatMaxN = 64;
struct MatArgs {
  const uint32_t* A;
  const uint32_t* B;
  uint32_t* C;       // may equal A
  uint64_t N;        // words per entry (a multiple of kb)
  uint32_t n, kb;    // matrix size; frequencies per workgroup (freq_matmul_block)
  uint32_t fold;     // products accumulated between folds (>= 1)
  uint32_t p, pinv;  // p < 2^31, p^-1 mod 2^32
  uint32_t r32;      // 2^32 mod p
  uint32_t kw, kws;  // K and floor(K 2^32 / p)
};
uint32_t freq_matmul_block(uint32_t n, uint64_t N);
hipError_t launch_freq_matmul(const MatArgs& a, hipStream_t stream);
// dst[r][t] = t < src_len ? src[r][t] : 0 for r < rows, t < dst_len; reduce_p != 0
// (< 2^31): every word reduced modulo reduce_p.
hipError_t launch_copy_rows(uint32_t* dst, uint64_t dst_stride, uint64_t dst_len, const uint32_t* src,
                            uint64_t src_stride, uint64_t src_len, uint32_t rows, hipStream_t stream,
                            uint32_t reduce_p = 0);

}  // namespace nttgpu
