// Types shared by the host library and the kernels (device-resident descriptors).
#pragma once
#include <stdint.h>

#include "arith.hpp"

namespace nttgpu {

// Per-(p, transform length) constants of the fused product (device memory).
// d = log2 N - m is the split depth: the product runs as 2^d sub-problems of length
// 2^m (section 5.1's Algorithm 1 with n1 = 2^d), each sub-problem h starting from the
// fold sum_k a[j + k 2^m] psi_h^k, psi_h = w_{2^d}^([h]_d).
//
// Truncation (the TFT of section 5.1 at sub-problem granularity): a product with
// lc <= lambda S coefficients needs only the sub-problems h < lambda = ceil(lc / S),
// the first lambda values of Algorithm 1's step-1 TFT of size 2^d.  The partials of
// the sub-problems h >= lambda are then fixed by the zero coefficients c_k = 0,
// k >= lambda, of every recombined position: u_miss = T u_known, with T the matrix
// below (entry (r, c) multiplies u_c into u_(lambda + r)).
template <typename T>
struct PolyConst {
  T p, p2, pinv, lazy;  // the arithmetic mode: 1 lazy ranges, 0 values below 2p, 2 doubles, p >= 2^49
  TwPair<T> fa[4][4];   // psi_h^k
  TwPair<T> fb[4][4];   // psi_h^k * sigma, sigma = 2^bits(T) / N mod p (Montgomery scale)
  TwPair<T> tft2[3];        // d = 2, lambda = 3: 1 x 3
  TwPair<T> tft3[3][3][7];  // d = 3, lambda = 5, 6, 7: (8 - lambda) x lambda
};

// One product in a fused launch.
struct FusedItem {
  const void* a;
  const void* b;
  void* c;
  uint64_t la, lb;
  const void* cst;  // PolyConst<T>
  const void* tw;   // TwPair<T>[2^LT]: forward universal table
  const void* twi;  // TwPair<T>[2^LT]: inverse universal table
  uint32_t log2n;
  uint32_t pad;
};

// Per-plan constants of a multi-pass transform of length 2^L = 2^L1 * 2^L2.
// Pass 1 (columns) transforms the 2^L2 strided vectors of length 2^L1 with the
// universal table; pass 2 (rows) twists row r (of length 2^L2) by G^j,
// G = w_N^([r]_L1), then transforms it (Algorithm 1, steps 2 and 3).  G^j =
// w_N^e with e = j [r]_L1 < N is read from two tables: w_N^e = lo[e & (2^B-1)] *
// hi[e >> B].  With 32-bit words the row pass reads them once per thread and row:
// for j = q + 2^10 c, G^j = G^q * w_(2^(L-10))^(c [r]_L1 mod 2^(L-10)), the second
// factor an entry of the universal table (same in every lane).
template <typename T>
struct PassConst {
  T p, p2, pinv, lazy;  // the arithmetic mode, as in PolyConst
  TwPair<T> ninv;     // n^-1
  TwPair<T> sigma;    // 2^bits(T) / N mod p
  TwPair<T> one;      // (1, floor(2^bits(T) / p)): Function 8 by 1 reduces any word to [0, 2p)
  uint32_t L, L1, L2, B;
  double rcp32;       // 2^32 / p rounded: estimates Shoup companions of 32-bit residues
  // Truncated transforms (section 5.1's TFT at row granularity):
  TwPair<T> sigma_row;    // 2^bits(T) / 2^L2 mod p: the Montgomery scale of a product
                          // whose row inverse is normalized and whose columns are
                          // inverted exactly (inverse TFT)
  T half;                 // (p + 1) / 2 = 2^-1 mod p
  TwPair<T> inv2pow[16];  // 2^-m mod p, m < 16: normalization of inverse sub-blocks
};

}  // namespace nttgpu
