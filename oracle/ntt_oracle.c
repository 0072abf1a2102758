/*
 * CPU oracle for exact NTT arithmetic over F_p, p = k*2^l + 1.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file; only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header, table or constant generator with the HIP path.
 *
 * Everything here is the plain mathematical definition, written for clarity:
 * residues are canonical in {0, ..., p-1} (section 2, storage convention), every
 * product is formed in unsigned __int128 and reduced with the C '%' operator, and
 * there is no lazy reduction, no precomputed-multiplicand trick, no blocking and no
 * fusion.  Residues are passed as uint64_t for every word size.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* (a * b) mod p by definition (section 2: "a rem b" of the long division). */
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t p) {
  return (uint64_t)(((u128)a * b) % p);
}

uint64_t orc_addmod(uint64_t a, uint64_t b, uint64_t p) {
  return (uint64_t)(((u128)a + b) % p);
}

uint64_t orc_submod(uint64_t a, uint64_t b, uint64_t p) {
  return (uint64_t)(((u128)a + p - b) % p);
}

/* a^e mod p by square-and-multiply. */
uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p, x = a % p;
  while (e) {
    if (e & 1) r = orc_mulmod(r, x, p);
    x = orc_mulmod(x, x, p);
    e >>= 1;
  }
  return r;
}

/* Inverse of a unit of F_p via Fermat (p prime). */
uint64_t orc_invmod(uint64_t a, uint64_t p) { return orc_powmod(a, p - 2, p); }

/*
 * FFT by its definition (section 5.1): out_i = sum_j w^(i*j) a_j, O(n^2).
 */
void orc_dft(uint64_t p, uint64_t w, const uint64_t* a, uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    uint64_t wi = orc_powmod(w, (uint64_t)i, p); /* w^i; the row's terms are (w^i)^j */
    uint64_t z = 1 % p;
    u128 acc = 0;
    for (size_t j = 0; j < n; ++j) {
      acc += (u128)orc_mulmod(z, a[j], p);
      if (acc >= ((u128)1 << 120)) acc %= p;
      z = orc_mulmod(z, wi, p);
    }
    out[i] = (uint64_t)(acc % p);
  }
}

/* One output of the transform: A(x) = sum_j a_j x^j by Horner's rule, O(n). */
uint64_t orc_horner(uint64_t p, const uint64_t* a, size_t n, uint64_t x) {
  uint64_t r = 0;
  for (size_t j = n; j-- > 0;) r = orc_addmod(orc_mulmod(r, x, p), a[j], p);
  return r;
}

static unsigned ilog2_exact(size_t n) {
  unsigned k = 0;
  while (((size_t)1 << k) < n) ++k;
  return k;
}

/* Bitwise mirror [i]_k of section 5.1. */
size_t orc_bitrev(size_t i, unsigned k) {
  size_t r = 0;
  for (unsigned b = 0; b < k; ++b) r |= ((i >> b) & 1u) << (k - 1 - b);
  return r;
}

/*
 * Textbook iterative radix-2 transform, natural order in and out, in place:
 * explicit bit-reversal permutation of the input, then log2(n) levels of
 * Cooley-Tukey butterflies (u, v) -> (u + z v, u - z v) with z running through the
 * powers of the level's root w^(n/len).  Computes out_i = sum_j w^(ij) a_j.
 */
void orc_ntt(uint64_t p, uint64_t w, uint64_t* a, size_t n) {
  unsigned k = ilog2_exact(n);
  for (size_t i = 0; i < n; ++i) {
    size_t r = orc_bitrev(i, k);
    if (i < r) { uint64_t t = a[i]; a[i] = a[r]; a[r] = t; }
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    uint64_t wl = orc_powmod(w, n / len, p);
    for (size_t start = 0; start < n; start += len) {
      uint64_t z = 1;
      for (size_t j = 0; j < len / 2; ++j) {
        uint64_t u = a[start + j];
        uint64_t v = orc_mulmod(z, a[start + j + len / 2], p);
        a[start + j] = orc_addmod(u, v, p);
        a[start + j + len / 2] = orc_submod(u, v, p);
        z = orc_mulmod(z, wl, p);
      }
    }
  }
}

/* Inverse: the transform with w^-1, then multiplication by n^-1, so inv(fwd(a)) = a. */
void orc_intt(uint64_t p, uint64_t w, uint64_t* a, size_t n) {
  orc_ntt(p, orc_invmod(w, p), a, n);
  uint64_t ninv = orc_invmod((uint64_t)(n % p), p);
  for (size_t i = 0; i < n; ++i) a[i] = orc_mulmod(a[i], ninv, p);
}

/*
 * Schoolbook product (section 5.2's problem): c_k = sum_{i+j=k} a_i b_j mod p for
 * k < la + lb - 1.  Word-size products are accumulated in 128 bits (reduced first
 * when p is wider than 32 bits, so the sum cannot overflow) and reduced once.
 */
void orc_polymul_schoolbook(uint64_t p, const uint64_t* a, size_t la, const uint64_t* b, size_t lb,
                            uint64_t* c) {
  if (la == 0 || lb == 0) return;
  size_t lc = la + lb - 1;
  int wide = p >= ((uint64_t)1 << 32);
  for (size_t k = 0; k < lc; ++k) {
    size_t i0 = k >= lb ? k - (lb - 1) : 0;
    size_t i1 = k < la ? k : la - 1;
    u128 acc = 0;
    for (size_t i = i0; i <= i1; ++i) {
      if (wide) {
        acc += (u128)orc_mulmod(a[i], b[k - i], p);
      } else {
        acc += (u128)a[i] * b[k - i];
      }
    }
    c[k] = (uint64_t)(acc % p);
  }
}

/*
 * Product through the transform (section 5.2): zero-pad both operands to the
 * transform length n >= la + lb - 1, two forward transforms, entry-wise product,
 * one inverse transform.  w must be a primitive n-th root of unity.
 */
int orc_polymul_ntt(uint64_t p, uint64_t w, size_t n, const uint64_t* a, size_t la, const uint64_t* b,
                    size_t lb, uint64_t* c) {
  if (la == 0 || lb == 0) return 0;
  if (la + lb - 1 > n) return -1;
  uint64_t* fa = (uint64_t*)calloc(n, sizeof(uint64_t));
  uint64_t* fb = (uint64_t*)calloc(n, sizeof(uint64_t));
  if (!fa || !fb) { free(fa); free(fb); return -5; }
  memcpy(fa, a, la * sizeof(uint64_t));
  memcpy(fb, b, lb * sizeof(uint64_t));
  orc_ntt(p, w, fa, n);
  orc_ntt(p, w, fb, n);
  for (size_t i = 0; i < n; ++i) fa[i] = orc_mulmod(fa[i], fb[i], p);
  orc_intt(p, w, fa, n);
  memcpy(c, fa, (la + lb - 1) * sizeof(uint64_t));
  free(fa);
  free(fb);
  return 0;
}

/*
 * Integer product by schoolbook on 16-bit limbs (little endian): C = A * B,
 * output limb j (32-bit) = floor(C / 2^(32 j)) mod 2^32 for j < ceil((na+nb)/2).
 * Column sums of 16x16-bit products are accumulated with a running 128-bit carry.
 */
void orc_intmul_schoolbook(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint32_t* c) {
  size_t nc16 = na + nb;
  size_t nc32 = (nc16 + 1) / 2;
  memset(c, 0, nc32 * sizeof(uint32_t));
  u128 carry = 0;
  for (size_t k = 0; k < nc16; ++k) {
    u128 col = carry;
    if (na && nb && k <= na + nb - 2) {
      size_t i0 = k >= nb ? k - (nb - 1) : 0;
      size_t i1 = k < na ? k : na - 1;
      for (size_t i = i0; i <= i1; ++i) col += (uint64_t)a[i] * b[k - i];
    }
    uint16_t limb = (uint16_t)(col & 0xFFFF);
    carry = col >> 16;
    c[k / 2] |= (uint32_t)limb << (16 * (k & 1));
  }
}

/*
 * Integer product by Kronecker segmentation and the three-prime transform
 * (section 5.3) with chunk size h = 16: the limbs are the coefficients of A(X), B(X)
 * with A(2^16) = a; C = A B is computed modulo p1, p2, p3 by orc_polymul_ntt, the
 * coefficients are rebuilt by Garner's mixed-radix CRT,
 *   x1 = r1, x2 = (r2 - x1) p1^-1 mod p2, x3 = (r3 - x1 - x2 p1) (p1 p2)^-1 mod p3,
 *   value = x1 + p1 x2 + p1 p2 x3,
 * and C(2^16) is evaluated with a sequential 128-bit carry.
 * roots[i] must be a primitive n-th root of unity mod primes[i]; n >= na + nb - 1.
 * Returns 0; -1 when min(na, nb) (2^16 - 1)^2 >= p1 p2 p3 (the coefficient bound of
 * section 5.3 would not determine the coefficients) or n < na + nb - 1.
 */
int orc_intmul_3prime(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint32_t* c,
                      const uint64_t* primes, const uint64_t* roots, size_t n) {
  size_t nc16 = na + nb;
  size_t nc32 = (nc16 + 1) / 2;
  memset(c, 0, nc32 * sizeof(uint32_t));
  if (na == 0 || nb == 0) return 0;
  size_t lc = na + nb - 1;
  {
    u128 bound = (u128)(na < nb ? na : nb) * 65535u * 65535u;
    u128 m = (u128)primes[0] * primes[1];
    /* bound >= m * p3  <=>  bound / m >= p3 (integer division is exact enough here) */
    if (bound / m >= primes[2]) return -1;
  }
  uint64_t* ra = (uint64_t*)malloc(na * sizeof(uint64_t));
  uint64_t* rb = (uint64_t*)malloc(nb * sizeof(uint64_t));
  uint64_t* r[3];
  for (int i = 0; i < 3; ++i) r[i] = (uint64_t*)malloc(lc * sizeof(uint64_t));
  for (size_t i = 0; i < na; ++i) ra[i] = a[i];
  for (size_t i = 0; i < nb; ++i) rb[i] = b[i];
  int rc = 0;
  for (int i = 0; i < 3 && rc == 0; ++i) rc = orc_polymul_ntt(primes[i], roots[i], n, ra, na, rb, nb, r[i]);
  uint64_t p1 = primes[0], p2 = primes[1], p3 = primes[2];
  uint64_t p1inv_p2 = orc_invmod(p1 % p2, p2);
  uint64_t p12inv_p3 = orc_invmod(orc_mulmod(p1 % p3, p2 % p3, p3), p3);
  u128 carry = 0;
  for (size_t k = 0; k < nc16 && rc == 0; ++k) {
    u128 value = 0;
    if (k < lc) {
      uint64_t x1 = r[0][k];
      uint64_t x2 = orc_mulmod(orc_submod(r[1][k], x1 % p2, p2), p1inv_p2, p2);
      uint64_t t = orc_submod(orc_submod(r[2][k], x1 % p3, p3), orc_mulmod(x2 % p3, p1 % p3, p3), p3);
      uint64_t x3 = orc_mulmod(t, p12inv_p3, p3);
      value = (u128)x1 + (u128)p1 * x2 + (u128)p1 * p2 * x3;
    }
    u128 col = carry + value;
    c[k / 2] |= (uint32_t)(col & 0xFFFF) << (16 * (k & 1));
    carry = col >> 16;
  }
  free(ra);
  free(rb);
  for (int i = 0; i < 3; ++i) free(r[i]);
  return rc;
}

/*
 * Garner digits of every coefficient: writes x1, x2, x3 for each of the lc residue
 * triples (used by the tests to check the bound value < p1 p2, i.e. x3 = 0).
 */
void orc_garner_digits(const uint64_t* r1, const uint64_t* r2, const uint64_t* r3, size_t lc,
                       const uint64_t* primes, uint64_t* x1, uint64_t* x2, uint64_t* x3) {
  uint64_t p1 = primes[0], p2 = primes[1], p3 = primes[2];
  uint64_t p1inv_p2 = orc_invmod(p1 % p2, p2);
  uint64_t p12inv_p3 = orc_invmod(orc_mulmod(p1 % p3, p2 % p3, p3), p3);
  for (size_t k = 0; k < lc; ++k) {
    x1[k] = r1[k];
    x2[k] = orc_mulmod(orc_submod(r2[k], r1[k] % p2, p2), p1inv_p2, p2);
    uint64_t t = orc_submod(orc_submod(r3[k], r1[k] % p3, p3), orc_mulmod(x2[k] % p3, p1 % p3, p3), p3);
    x3[k] = orc_mulmod(t, p12inv_p3, p3);
  }
}

/* Element-wise helpers over arrays (kept for the tests' convenience). */
void orc_mulmod_vec(uint64_t p, const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; ++i) out[i] = orc_mulmod(a[i], b[i], p);
}

/*
 * Polynomial matrix product (section 5.2): C = A B for n x n matrices over F_p[x]
 * whose entries have degree < d.  Entry (i, j) of C is sum_l A_il B_lj, the products
 * of polynomials written out coefficient by coefficient:
 *   C_ij[k] = sum_l sum_{s + t = k} A_il[s] B_lj[t]  mod p,  k < 2d - 1.
 * Layout: entry (i, j) of A and B at (i n + j) d, of C at (i n + j)(2d - 1).
 */
uint64_t orc_polymatmul_coeff(uint64_t p, size_t n, const uint64_t* A, const uint64_t* B, size_t d, size_t i,
                              size_t j, size_t k) {
  u128 acc = 0;
  const size_t s0 = k >= d ? k - (d - 1) : 0;
  const size_t s1 = k < d ? k : d - 1;
  for (size_t l = 0; l < n; ++l) {
    const uint64_t* a = A + (i * n + l) * d;
    const uint64_t* b = B + (l * n + j) * d;
    for (size_t s = s0; s <= s1; ++s) {
      acc += (u128)orc_mulmod(a[s], b[k - s], p);
      if (acc >> 120) acc %= p;
    }
  }
  return (uint64_t)(acc % p);
}

void orc_polymatmul(uint64_t p, size_t n, const uint64_t* A, const uint64_t* B, size_t d, uint64_t* C) {
  if (n == 0 || d == 0) return;
  const size_t lc = 2 * d - 1;
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j)
      for (size_t k = 0; k < lc; ++k) C[(i * n + j) * lc + k] = orc_polymatmul_coeff(p, n, A, B, d, i, j, k);
}

void orc_horner_many(uint64_t p, const uint64_t* a, size_t n, const uint64_t* xs, uint64_t* out, size_t m) {
  for (size_t i = 0; i < m; ++i) out[i] = orc_horner(p, a, n, xs[i]);
}

/* C mod q for a little-endian 32-bit limb vector (q < 2^63). */
uint64_t orc_limbs32_mod(const uint32_t* x, size_t n, uint64_t q) {
  u128 r = 0;
  for (size_t j = n; j-- > 0;) r = ((r << 32) + x[j]) % q;
  return (uint64_t)r;
}

uint64_t orc_limbs16_mod(const uint16_t* x, size_t n, uint64_t q) {
  u128 r = 0;
  for (size_t j = n; j-- > 0;) r = ((r << 16) + x[j]) % q;
  return (uint64_t)r;
}
