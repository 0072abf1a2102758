// Host side of the library: number theory, plan tables, argument checking and the
// launch sequences behind the C ABI of include/ntt_mi355x.h.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ntt_mi355x.h"
#include "arith_apply.hpp"
#include "kernels.hpp"

using namespace nttgpu;

typedef unsigned __int128 u128;

// ============================================================================ errors
namespace {
thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return NTT_OK;
}

// Set between ntt_graph_begin and ntt_graph_end on the capturing thread: calls that
// would allocate, copy from the host or wait are refused meanwhile.
thread_local bool g_capturing = false;

bool capturing(hipStream_t s) {
  if (g_capturing) return true;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

// ============================================================================ tuning choices
// Values chosen by the autotuner (or set by hand) that override the built-in
// defaults.  Keys:
//   split.w<W>.L<L>   row length 2^L2 of two-pass transform plans of length 2^L
//   psplit.w<W>.L<L>  the same for the plans the products use
//   fused.single.max.w<W>  largest log2 N of a single product served by the fused
//                     one-workgroup kernel
//   single.split.w<W>.L<L>  split depth d of a single product of length 2^L over 2^d
//                     workgroups (0: not split)
//   tft.rows.w<W>     two-pass products truncated at row granularity (1) or transformed at
//                     full length (0, the default)
//   server.copy_threads  host copy threads of a serving loop created afterwards
std::mutex g_tune_mu;
std::map<std::string, int64_t> g_tune;

// Range check of one (key, value); returns false for an unknown key or a value the
// kernels do not implement.
bool tune_valid(const std::string& key, int64_t v) {
  int w = 0, L = 0;
  char tail = 0;
  if (sscanf(key.c_str(), "split.w%d.L%d%c", &w, &L, &tail) == 2 ||
      sscanf(key.c_str(), "psplit.w%d.L%d%c", &w, &L, &tail) == 2) {
    if (w == 32) return L >= 15 && L <= 26 && v >= 12 && v <= 14;
    if (w == 64) return L >= 14 && L <= 26 && v >= 12 && v <= 13;
    return false;
  }
  if (sscanf(key.c_str(), "single.split.w%d.L%d%c", &w, &L, &tail) == 2) {
    if (w != 32 && w != 64) return false;
    if (L < 11 || L > fused_max_log2n(w)) return false;
    return v == 0 || split_supported(w, L, (int)v);
  }
  if (sscanf(key.c_str(), "tft.rows.w%d%c", &w, &tail) == 1) return (w == 32 || w == 64) && (v == 0 || v == 1);
  if (key == "server.copy_threads") return v >= 0 && v <= 63;
  if (key == "batch.fork") return v == 0 || v == 1;
  if (key == "fused.m15.w32") return v == 0 || v == 1;
  if (key == "server.batches_per_stream") return v >= 1 && v <= 8;
  if (sscanf(key.c_str(), "fused.single.max.w%d%c", &w, &tail) == 1) {
    if (w == 32) return v >= 14 && v <= 16;
    if (w == 64) return v >= 13 && v <= 15;
  }
  return false;
}

int64_t tune_value(const std::string& key, int64_t dflt) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  return it == g_tune.end() ? dflt : it->second;
}

std::string tune_key(const char* prefix, int wb, int L) {
  char buf[64];
  if (L >= 0) snprintf(buf, sizeof(buf), "%s.w%d.L%d", prefix, wb, L);
  else snprintf(buf, sizeof(buf), "%s.w%d", prefix, wb);
  return buf;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(NTT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ============================================================================ number theory
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

// Miller-Rabin with the first twelve prime bases: deterministic for all n < 2^64.
bool is_prime_u64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : bases)
    if (n % b == 0) return n == b;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t b : bases) {
    uint64_t x = powmod(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int i = 1; i < s; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        composite = false;
        break;
      }
    }
    if (composite) return false;
  }
  return true;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Pollard-Brent rho: a nontrivial factor of the composite odd n.
uint64_t rho_factor(uint64_t n) {
  for (uint64_t c = 1;; ++c) {
    uint64_t y = 2, x = 2, g = 1, q = 1, ys = 2;
    uint64_t r = 1;
    const uint64_t m = 128;
    auto f = [&](uint64_t v) { return (mulmod(v, v, n) + c) % n; };
    do {
      x = y;
      for (uint64_t i = 0; i < r; ++i) y = f(y);
      uint64_t k = 0;
      do {
        ys = y;
        for (uint64_t i = 0; i < std::min(m, r - k); ++i) {
          y = f(y);
          q = mulmod(q, x > y ? x - y : y - x, n);
        }
        g = gcd_u64(q, n);
        k += m;
      } while (k < r && g == 1);
      r <<= 1;
    } while (g == 1);
    if (g == n) {
      do {
        ys = f(ys);
        g = gcd_u64(x > ys ? x - ys : ys - x, n);
      } while (g == 1);
    }
    if (g != n) return g;
  }
}

void factor_into(uint64_t n, std::vector<uint64_t>& out) {
  if (n == 1) return;
  for (uint64_t q = 2; q < 1000 && q * q <= n; ++q) {
    if (n % q == 0) {
      out.push_back(q);
      while (n % q == 0) n /= q;
    }
  }
  if (n == 1) return;
  if (is_prime_u64(n)) {
    out.push_back(n);
    return;
  }
  uint64_t f = rho_factor(n);
  factor_into(f, out);
  factor_into(n / f, out);
}

std::vector<uint64_t> distinct_prime_factors(uint64_t n) {
  std::vector<uint64_t> f;
  factor_into(n, f);
  std::sort(f.begin(), f.end());
  f.erase(std::unique(f.begin(), f.end()), f.end());
  return f;
}

bool generates(uint64_t g, uint64_t p, const std::vector<uint64_t>& qs) {
  if (g % p == 0) return false;
  for (uint64_t q : qs)
    if (powmod(g, (p - 1) / q, p) == 1) return false;
  return true;
}

uint64_t smallest_generator(uint64_t p) {
  const std::vector<uint64_t> qs = distinct_prime_factors(p - 1);
  for (uint64_t g = 2; g < p; ++g)
    if (generates(g, p, qs)) return g;
  return 0;
}

int two_adic_order(uint64_t p) {
  uint64_t k = p - 1;
  int l = 0;
  while (k && (k & 1) == 0) {
    k >>= 1;
    ++l;
  }
  return l;
}

uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }

uint32_t brev(uint32_t i, int k) {
  uint32_t r = 0;
  for (int b = 0; b < k; ++b) r |= ((i >> b) & 1u) << (k - 1 - b);
  return r;
}

int ceil_log2(uint64_t n) {
  int L = 0;
  while ((1ull << L) < n) ++L;
  return L;
}

// ============================================================================ tables
constexpr int kUniversalMaxLog = 16;

template <typename T>
TwPair<T> pair_of(uint64_t w, uint64_t p) {
  TwPair<T> t;
  t.w = (T)w;
  if constexpr (std::is_same<T, double>::value) t.ws = (double)w / (double)p;  // not read by the FP64 product
  else t.ws = (T)(((u128)w << (8 * sizeof(T))) / p);
  return t;
}

// Universal bit-reversed tables: tw[2^s + i] = w_{2^(s+1)}^([i]_s) for s < LT.
template <typename T>
void build_universal(uint64_t p, uint64_t g, int LT, bool inverse, std::vector<TwPair<T>>& out) {
  out.assign((size_t)1 << LT, pair_of<T>(1, p));
  std::vector<uint64_t> pw;
  for (int s = 0; s < LT; ++s) {
    uint64_t w = powmod(g, (p - 1) >> (s + 1), p);
    if (inverse) w = invmod(w, p);
    pw.assign((size_t)1 << s, 1);
    for (size_t e = 1; e < pw.size(); ++e) pw[e] = mulmod(pw[e - 1], w, p);
    for (uint32_t i = 0; i < (1u << s); ++i) out[((size_t)1 << s) + i] = pair_of<T>(pw[brev(i, s)], p);
  }
}

template <typename T>
void build_powers(uint64_t base, uint64_t p, size_t n, uint64_t scale, std::vector<TwPair<T>>& out) {
  out.resize(n);
  uint64_t x = scale % p;
  for (size_t e = 0; e < n; ++e) {
    out[e] = pair_of<T>(x, p);
    x = mulmod(x, base, p);
  }
}

uint64_t inv_pow2_word(uint64_t p, int bits) {  // p^-1 mod 2^bits by Newton iteration
  uint64_t x = p;  // correct to 3 bits for odd p
  for (int i = 0; i < 6; ++i) x *= 2 - p * x;
  if (bits == 32) x &= 0xFFFFFFFFull;
  return x;
}

}  // namespace

// ============================================================================ plan
struct ntt_plan {
  uint64_t p, g, w, winv, ninv;
  uint32_t log2n, wbits, flags, passes, L1, L2, B, LT;
  int device;
  int mode;      // the kernels' arithmetic mode: 1 lazy ranges, 0 below 2p, 2 doubles with p >= 2^49
  bool numeric;  // residues held in doubles (FP64 arithmetic), p < 2^50
  void* dmem;
  size_t dbytes;
  const void *tw, *twi, *tlo, *thi, *tilo, *tihi, *tihin, *tihin1, *polyc, *passc;
};

namespace {

struct Blob {
  std::vector<unsigned char> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = (bytes.size() + 255) & ~(size_t)255;
    bytes.resize(off + n);
    memcpy(bytes.data() + off, src, n);
    return off;
  }
};

template <typename T>
int build_plan_tables(ntt_plan* pl) {
  const uint64_t p = pl->p;
  const int L = (int)pl->log2n;
  const int W = (int)(8 * sizeof(T));
  Blob blob;
  std::vector<TwPair<T>> tw, twi;
  // long two-pass transforms also read w_(2^(L-10)) powers from the table
  pl->LT = (uint32_t)std::max(1, std::min(L, std::max(kUniversalMaxLog, L - 10)));
  build_universal<T>(p, pl->g, (int)pl->LT, false, tw);
  build_universal<T>(p, pl->g, (int)pl->LT, true, twi);
  const size_t o_tw = blob.add(tw.data(), tw.size() * sizeof(TwPair<T>));
  const size_t o_twi = blob.add(twi.data(), twi.size() * sizeof(TwPair<T>));

  const uint64_t N = 1ull << L;
  // the scale the entry-wise product removes: 2^W / N for Montgomery's product over
  // W-bit words, 1 / N for the FP64 product (no Montgomery factor)
  constexpr bool kNumeric = std::is_same<T, double>::value;
  const uint64_t sigma = kNumeric ? pl->ninv : mulmod((uint64_t)((((u128)1) << W) % p), pl->ninv, p);
  const T pinv_word = kNumeric ? (T)(1.0 / (double)p) : (T)inv_pow2_word(p, W);

  // Fused-product constants.
  PolyConst<T> pc;
  memset(&pc, 0, sizeof(pc));
  pc.p = (T)p;
  pc.p2 = (T)(2 * p);
  pc.pinv = pinv_word;
  pc.lazy = (T)pl->mode;
  {
    const int lmax = (W == 32) ? 14 : 13;
    const int d = L > lmax ? L - lmax : 0;
    const uint64_t root_d = powmod(pl->g, (p - 1) >> d, p);  // w_{2^d}
    for (int h = 0; h < 4; ++h) {
      const uint64_t psi = (h < (1 << d)) ? powmod(root_d, brev((uint32_t)h, d), p) : 1;
      uint64_t x = 1;
      for (int k = 0; k < 4; ++k) {
        pc.fa[h][k] = pair_of<T>(x, p);
        pc.fb[h][k] = pair_of<T>(mulmod(x, sigma, p), p);
        x = mulmod(x, psi, p);
      }
    }
  }
  {
    // completion of truncated products (d = 2 and 3): the recombination map W of the
    // last d inverse stages (TWI[2^t + blk]), then T = -A^-1 B with A = W[k >= lam][h >= lam],
    // B = W[k >= lam][h < lam]
    const int K8 = (int)std::min<size_t>(twi.size(), 8);
    for (int d = 2; d <= 3 && (1 << d) <= K8; ++d) {
      const int n = 1 << d;
      std::vector<std::vector<uint64_t>> W(n, std::vector<uint64_t>(n, 0));
      for (int hcol = 0; hcol < n; ++hcol) {
        std::vector<uint64_t> u(n, 0);
        u[hcol] = 1;
        for (int t = d - 1; t >= 0; --t) {
          const int half = 1 << (d - 1 - t);
          for (int blk = 0; blk < (1 << t); ++blk) {
            const uint64_t w = (uint64_t)twi[(1 << t) + blk].w;
            for (int i = 0; i < half; ++i) {
              const int x = blk * 2 * half + i, y = x + half;
              const uint64_t X = u[x], Y = u[y];
              u[x] = (X + Y) % p;
              u[y] = mulmod((X + p - Y) % p, w, p);
            }
          }
        }
        for (int k = 0; k < n; ++k) W[k][hcol] = u[k];
      }
      for (int lam = n / 2 + 1; lam < n; ++lam) {
        const int m = n - lam;
        // augmented [A | B], solved in place by Gauss-Jordan elimination mod p
        std::vector<std::vector<uint64_t>> G(m, std::vector<uint64_t>(m + lam, 0));
        for (int r = 0; r < m; ++r) {
          for (int cidx = 0; cidx < m; ++cidx) G[r][cidx] = W[lam + r][lam + cidx];
          for (int cidx = 0; cidx < lam; ++cidx) G[r][m + cidx] = W[lam + r][cidx];
        }
        bool ok_solve = true;
        for (int col = 0; col < m && ok_solve; ++col) {
          int piv = -1;
          for (int r = col; r < m; ++r)
            if (G[r][col]) { piv = r; break; }
          if (piv < 0) { ok_solve = false; break; }
          std::swap(G[piv], G[col]);
          const uint64_t inv = invmod(G[col][col], p);
          for (auto& e : G[col]) e = mulmod(e, inv, p);
          for (int r = 0; r < m; ++r) {
            if (r == col || !G[r][col]) continue;
            const uint64_t f = G[r][col];
            for (int cidx = 0; cidx < m + lam; ++cidx) G[r][cidx] = (G[r][cidx] + p - mulmod(f, G[col][cidx], p)) % p;
          }
        }
        if (!ok_solve) return fail(NTT_EDEVICE, "truncated-product completion matrix is singular (p = %llu, d = %d)",
                                   (unsigned long long)p, d);
        for (int r = 0; r < m; ++r)
          for (int cidx = 0; cidx < lam; ++cidx) {
            const uint64_t tv = (p - G[r][m + cidx]) % p;  // T = -A^-1 B
            if (d == 2) pc.tft2[cidx] = pair_of<T>(tv, p);
            else pc.tft3[lam - 5][r][cidx] = pair_of<T>(tv, p);
          }
      }
    }
  }
  const size_t o_pc = blob.add(&pc, sizeof(pc));

  // Two-pass constants and twist tables.
  PassConst<T> sc;
  memset(&sc, 0, sizeof(sc));
  sc.p = (T)p;
  sc.p2 = (T)(2 * p);
  sc.pinv = pinv_word;
  sc.lazy = (T)pl->mode;
  sc.ninv = pair_of<T>(pl->ninv, p);
  sc.sigma = pair_of<T>(sigma, p);
  sc.one = pair_of<T>(1, p);
  sc.L = (uint32_t)L;
  sc.L1 = pl->L1;
  sc.L2 = pl->L2;
  sc.B = pl->B;
  sc.rcp32 = 4294967296.0 / (double)p;
  {
    // truncated transforms: the row inverse is normalized by 2^-L2 (the product's
    // Montgomery scale 2^W / 2^L2, 1 / 2^L2 for doubles) and sub-blocks by 2^-m
    const uint64_t inv2 = (p + 1) / 2;
    uint64_t pw = 1;
    for (int m = 0; m < 16; ++m) {
      sc.inv2pow[m] = pair_of<T>(pw, p);
      pw = mulmod(pw, inv2, p);
    }
    const uint64_t inv_n1 = powmod(inv2, pl->passes > 1 ? pl->L2 : (uint32_t)L, p);
    const uint64_t rw = kNumeric ? 1 : (uint64_t)((((u128)1) << W) % p);
    sc.sigma_row = pair_of<T>(mulmod(rw, inv_n1, p), p);
    sc.half = (T)inv2;
  }
  const size_t o_sc = blob.add(&sc, sizeof(sc));
  size_t o_lo = 0, o_hi = 0, o_ilo = 0, o_ihi = 0, o_ihin = 0, o_ihin1 = 0;
  if (pl->passes > 1) {
    const int B = (int)pl->B;
    std::vector<TwPair<T>> lo, hi, ilo, ihi, ihin, ihin1;
    build_powers<T>(pl->w, p, (size_t)1 << B, 1, lo);
    build_powers<T>(powmod(pl->w, 1ull << B, p), p, (size_t)1 << (L - B), 1, hi);
    build_powers<T>(pl->winv, p, (size_t)1 << B, 1, ilo);
    build_powers<T>(powmod(pl->winv, 1ull << B, p), p, (size_t)1 << (L - B), 1, ihi);
    build_powers<T>(powmod(pl->winv, 1ull << B, p), p, (size_t)1 << (L - B), pl->ninv, ihin);
    // the inverse twist with 2^-L2: normalized row inverses (inverse truncated transform)
    build_powers<T>(powmod(pl->winv, 1ull << B, p), p, (size_t)1 << (L - B), powmod((p + 1) / 2, pl->L2, p), ihin1);
    o_lo = blob.add(lo.data(), lo.size() * sizeof(TwPair<T>));
    o_hi = blob.add(hi.data(), hi.size() * sizeof(TwPair<T>));
    o_ilo = blob.add(ilo.data(), ilo.size() * sizeof(TwPair<T>));
    o_ihi = blob.add(ihi.data(), ihi.size() * sizeof(TwPair<T>));
    o_ihin = blob.add(ihin.data(), ihin.size() * sizeof(TwPair<T>));
    o_ihin1 = blob.add(ihin1.data(), ihin1.size() * sizeof(TwPair<T>));
  }
  (void)N;
  void* d = nullptr;
  if (hipMalloc(&d, blob.bytes.size()) != hipSuccess)
    return fail(NTT_ENOMEM, "hipMalloc of %zu bytes of plan tables failed", blob.bytes.size());
  if (hipMemcpy(d, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return fail(NTT_EDEVICE, "upload of plan tables failed");
  }
  unsigned char* base = (unsigned char*)d;
  pl->dmem = d;
  pl->dbytes = blob.bytes.size();
  pl->tw = base + o_tw;
  pl->twi = base + o_twi;
  pl->polyc = base + o_pc;
  pl->passc = base + o_sc;
  pl->tlo = pl->passes > 1 ? base + o_lo : nullptr;
  pl->thi = pl->passes > 1 ? base + o_hi : nullptr;
  pl->tilo = pl->passes > 1 ? base + o_ilo : nullptr;
  pl->tihi = pl->passes > 1 ? base + o_ihi : nullptr;
  pl->tihin = pl->passes > 1 ? base + o_ihin : nullptr;
  pl->tihin1 = pl->passes > 1 ? base + o_ihin1 : nullptr;
  return NTT_OK;
}

const uint64_t kMaxModulus = 1ull << 62;

int check_modulus(uint64_t p, int* l_out) {
  if (p < 3 || p >= kMaxModulus) return fail(NTT_EUNSUPPORTED, "modulus %llu outside [3, 2^62)", (unsigned long long)p);
  // the last modulus found prime (a batch names the same few primes many times)
  static thread_local uint64_t last_prime = 0;
  if (p != last_prime) {
    if (!is_prime_u64(p)) return fail(NTT_ENOTPRIME, "modulus %llu is not prime", (unsigned long long)p);
    last_prime = p;
  }
  *l_out = two_adic_order(p);
  return NTT_OK;
}

int create_plan(ntt_plan** out, uint64_t p, uint64_t g, uint32_t log2n, uint32_t flags, bool product = false,
                bool numeric = false) {
  if (g_capturing)
    return fail(NTT_EINVAL, "plan for p = %llu, N = 2^%u does not exist yet and cannot be created during a graph "
                "capture: run the call once before capturing it", (unsigned long long)p, log2n);
  int l = 0;
  int rc = check_modulus(p, &l);
  if (rc) return rc;
  if (log2n > 26) return fail(NTT_EUNSUPPORTED, "log2n = %u exceeds 26", log2n);
  if ((int)log2n > l)
    return fail(NTT_ENOROOT, "2^%u does not divide p - 1 (2-adic order %d)", log2n, l);
  if (flags & ~(NTT_BITREV_OUT | NTT_BITREV_IN | NTT_VALIDATE | NTT_FP64))
    return fail(NTT_EINVAL, "unknown flags 0x%x", flags);
  if (flags & NTT_FP64) numeric = true;
  if (numeric && p >= (1ull << 50))
    return fail(NTT_EUNSUPPORTED, "FP64 residues need p < 2^50 (p = %llu)", (unsigned long long)p);
  if (numeric && (flags & NTT_VALIDATE)) return fail(NTT_EUNSUPPORTED, "NTT_VALIDATE checks integer words, not doubles");
  if (g == 0) {
    g = smallest_generator(p);
  } else if (!generates(g, p, distinct_prime_factors(p - 1))) {
    return fail(NTT_ENOROOT, "%llu does not generate F_p^*", (unsigned long long)g);
  }
  ntt_plan* pl = new (std::nothrow) ntt_plan();
  if (!pl) return fail(NTT_ENOMEM, "host allocation failed");
  pl->p = p;
  pl->g = g;
  pl->log2n = log2n;
  pl->flags = flags;
  pl->numeric = numeric;
  pl->wbits = (p < (1ull << 31) && !numeric) ? 32 : 64;
  // arithmetic mode of the kernels (kLazy 1, kSafe 0, kBand 2: see the butterflies)
  pl->mode = numeric ? (p < (1ull << 48) ? 1 : p < (1ull << 49) ? 0 : 2) : (pl->wbits == 64 || p < (1ull << 30) ? 1 : 0);
  pl->w = powmod(g, (p - 1) >> log2n, p);
  pl->winv = invmod(pl->w, p);
  pl->ninv = invmod((1ull << log2n) % p, p);
  const int wb = (int)pl->wbits;
  if ((int)log2n <= lds_max_log2n(wb)) {
    pl->passes = 1;
    pl->L1 = 0;
    pl->L2 = log2n;
  } else {
    pl->passes = 2;
    pl->L2 = (uint32_t)tune_value(tune_key(product ? "psplit" : "split", wb, (int)log2n), pass_max_row_log2(wb));
    pl->L1 = log2n - pl->L2;
  }
  if (numeric && pl->passes > 1 && pl->L1 > 10) {
    delete pl;
    return fail(NTT_EUNSUPPORTED, "FP64 transforms of length 2^%u: columns of 2^%u words exceed 2^10", log2n,
                log2n - (uint32_t)pass_max_row_log2(wb));
  }
  pl->B = (log2n + 1) / 2;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    delete pl;
    return fail(NTT_EDEVICE, "hipGetDevice failed");
  }
  rc = numeric ? build_plan_tables<double>(pl)
               : (pl->wbits == 32 ? build_plan_tables<uint32_t>(pl) : build_plan_tables<uint64_t>(pl));
  if (rc) {
    delete pl;
    return rc;
  }
  *out = pl;
  return NTT_OK;
}

// ============================================================================ per-device context
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

struct DeviceCtx {
  std::mutex mu;
  // Fork streams of batch calls (class Fork): kForkLanes per caller stream, for the
  // kForkCallers caller streams used most recently (a bounded set: callers' streams come
  // and go, these are never destroyed); an older caller's lanes pass to a new caller.
  struct Lanes {
    std::vector<hipStream_t> s;
    uint64_t used = 0;
  };
  std::map<hipStream_t, Lanes> lanes;
  uint64_t lane_clock = 0;
  std::map<std::pair<uint64_t, uint32_t>, ntt_plan*> plans;
  Staging ring[8];
  unsigned next = 0;
  int cus = 0;
  uint32_t* flag = nullptr;
};

std::mutex g_ctx_mu;
std::map<int, DeviceCtx*> g_ctx;

DeviceCtx* device_ctx(int dev) {
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) return it->second;
  DeviceCtx* c = new DeviceCtx();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  c->cus = cus;
  g_ctx[dev] = c;
  return c;
}

// Cached plan for (current device, p, log2n) with the smallest generator.
// product: the plan's two-pass row length is the one tuned for products (whose row
// pass is the fused row product); otherwise the one tuned for transforms.  Each kind
// has its own cache key (p < 2^62, so bits 62 and 63 are free).
// create = false: only look the plan up (callers that must not allocate).
int cached_plan(uint64_t p, uint32_t log2n, ntt_plan** out, bool numeric = false, bool product = true,
                bool create = true) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NTT_EDEVICE, "hipGetDevice failed");
  DeviceCtx* c = device_ctx(dev);
  std::lock_guard<std::mutex> lk(c->mu);
  const uint64_t tag = (numeric ? (1ull << 63) : 0) | (product ? 0 : (1ull << 62));
  auto key = std::make_pair(p | tag, log2n);
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    *out = it->second;
    return NTT_OK;
  }
  if (!create)
    return fail(NTT_EINVAL, "no cached plan for p = %llu and transform length 2^%u on device %d: one polymul_modp "
                "call with this modulus and transform length creates it", (unsigned long long)p, log2n, dev);
  ntt_plan* pl = nullptr;
  int rc = create_plan(&pl, p, 0, log2n, NTT_BITREV_OUT | NTT_BITREV_IN, product, numeric);
  if (rc) return rc;
  c->plans[key] = pl;
  *out = pl;
  return NTT_OK;
}

// Copies `bytes` of host data into device memory `dst` on `stream` through a pinned
// staging slot; the slot is reused only after the copy that used it has completed.
int upload(DeviceCtx* c, void* dst, const void* src, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return NTT_OK;
  if (capturing(stream))
    return fail(NTT_EINVAL, "this call copies host descriptors and cannot be captured in a graph: "
                "use a polymul_batch_create handle");
  std::lock_guard<std::mutex> lk(c->mu);
  Staging& s = c->ring[c->next++ % 8];
  if (s.pending) {
    HIP_TRY(hipEventSynchronize(s.ev));
    s.pending = false;
  }
  if (!s.ev) HIP_TRY(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
  if (s.cap < bytes) {
    if (s.host) HIP_TRY(hipHostFree(s.host));
    s.host = nullptr;
    size_t cap = std::max(bytes, (size_t)65536);
    HIP_TRY(hipHostMalloc(&s.host, cap, hipHostMallocDefault));
    s.cap = cap;
  }
  memcpy(s.host, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(s.ev, stream));
  s.pending = true;
  return NTT_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned_to(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// Synchronous check that every element of `batch` vectors is < p (NTT_VALIDATE).
int validate_range(int wb, const void* x, size_t n, size_t stride, size_t batch, uint64_t p, hipStream_t stream) {
  if (capturing(stream)) return fail(NTT_EINVAL, "NTT_VALIDATE waits for the device and cannot be captured in a graph");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceCtx* c = device_ctx(dev);
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->flag) HIP_TRY(hipMalloc((void**)&c->flag, sizeof(uint32_t)));
  HIP_TRY(launch_fill_u32(c->flag, 1, 0u, stream));
  HIP_TRY(launch_range_check(wb, x, n, stride, (uint32_t)batch, p, c->flag, stream));
  uint32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->flag, sizeof(h), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (h) return fail(NTT_ERANGE, "input holds a value >= p = %llu", (unsigned long long)p);
  return NTT_OK;
}

// ---------------------------------------------------------------------------- transforms
int run_transform(const ntt_plan* pl, bool inverse, const void* in, void* out, size_t batch, size_t stride,
                  void* ws, size_t wsb, hipStream_t stream) {
  if (!pl) return fail(NTT_EINVAL, "plan is NULL");
  const size_t n = (size_t)1 << pl->log2n;
  const size_t esz = pl->wbits / 8;
  if (batch == 0) return ok();
  if (!in || !out) return fail(NTT_EINVAL, "NULL vector pointer");
  if (!aligned_to(in, esz) || !aligned_to(out, esz)) return fail(NTT_EINVAL, "vectors must be %zu-byte aligned", esz);
  if (stride < n) return fail(NTT_EINVAL, "stride %zu < n = %zu", stride, n);
  if (batch > 0xFFFFFFFFull) return fail(NTT_EINVAL, "batch too large");
  const size_t need = ntt_workspace_bytes(pl, batch);
  if (wsb < need || (need && !ws)) return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, wsb);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != pl->device) return fail(NTT_EINVAL, "plan belongs to device %d, current device is %d", pl->device, dev);
  const int wb = pl->numeric ? kWordF64 : (int)pl->wbits;  // kernel word code
  if (pl->flags & NTT_VALIDATE) {
    int rc = validate_range(wb, in, n, stride, batch, pl->p, stream);
    if (rc) return rc;
  }
  if (pl->passes == 1) {
    LdsNttArgs a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.stride = stride;
    a.pc = pl->passc;
    a.tw = pl->tw;
    a.twi = pl->twi;
    a.L = pl->log2n;
    a.bitrev = inverse ? ((pl->flags & NTT_BITREV_IN) ? 1 : 0) : ((pl->flags & NTT_BITREV_OUT) ? 1 : 0);
    a.batch = (uint32_t)batch;
    HIP_TRY(launch_lds_ntt(wb, inverse, a, stream));
    return ok();
  }
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.pc = pl->passc;
  a.tw = pl->tw;
  a.twi = pl->twi;
  a.tlo = pl->tlo;
  a.thi = pl->thi;
  a.tilo = pl->tilo;
  a.tihi = pl->tihin;  // the inverse transform includes n^-1
  a.batch = (uint32_t)batch;
  a.valid = n;
  const int L1 = (int)pl->L1, L2 = (int)pl->L2;
  if (!inverse) {
    const bool natural = !(pl->flags & NTT_BITREV_OUT);
    void* X = natural ? ws : out;
    const size_t xs = natural ? n : stride;
    a.in = in;
    a.in_stride = stride;
    a.out = X;
    a.out_stride = xs;
    HIP_TRY(launch_col_fwd(wb, a, L1, L2, stream));
    a.in = X;
    a.in_stride = xs;
    HIP_TRY(launch_row_fwd(wb, a, L1, L2, stream));
    if (natural) HIP_TRY(launch_bitrev_permute(wb, X, out, xs, stride, pl->log2n, (uint32_t)batch, stream));
  } else {
    const bool natural = !(pl->flags & NTT_BITREV_IN);
    const void* src = in;
    size_t ss = stride;
    if (natural) {
      HIP_TRY(launch_bitrev_permute(wb, in, ws, stride, n, pl->log2n, (uint32_t)batch, stream));
      src = ws;
      ss = n;
    }
    a.in = src;
    a.in_stride = ss;
    a.out = natural ? ws : out;
    a.out_stride = natural ? n : stride;
    HIP_TRY(launch_row_inv(wb, a, L1, L2, true, stream));
    a.in = a.out;
    a.in_stride = a.out_stride;
    a.out = out;
    a.out_stride = stride;
    HIP_TRY(launch_col_inv(wb, a, L1, L2, stream));
  }
  return ok();
}

}  // namespace

// ---------------------------------------------------------------------------- truncated transforms
// Section 5.1's TFT.  Two-pass plans truncate at row granularity (Algorithm 1 with n1 =
// 2^L2: only the first lambda rows of step 3 run) on the wave kernels' shapes.
bool tft_rows_ok(const ntt_plan* pl) {
  if (pl->passes == 1) return true;
  if (pl->L1 > 10) return false;
  return pl->wbits == 32 ? (pl->L2 >= 12 && pl->L2 <= 14) : (pl->L2 >= 12 && pl->L2 <= 13);
}

template <typename T>
TftArgs tft_args(const ntt_plan* pl) {
  TftArgs a;
  memset(&a, 0, sizeof(a));
  a.pc = pl->passc;
  a.tw = pl->tw;
  a.twi = pl->twi;
  a.tlo = pl->tlo;
  a.thi = pl->thi;
  a.tilo = pl->tilo;
  a.tihi = pl->tihi;  // the inverse TFT is normalized: no n^-1 in the untwist
  a.L = pl->log2n;
  a.L1 = pl->L1;
  a.L2 = pl->L2;
  return a;
}

size_t tft_ws_bytes(const ntt_plan* pl, size_t batch) {
  if (!pl || pl->passes == 1) return 0;
  // one row-major copy of every vector (at most all 2^L1 rows) and one row buffer
  return align256(((size_t)1 << pl->log2n) * (pl->wbits / 8) * batch) + align256(((size_t)1 << pl->L2) * (pl->wbits / 8) * batch);
}

int tft_check(const ntt_plan* pl, const void* in, void* out, size_t batch, size_t ws_bytes, void* ws, bool* done) {
  *done = false;
  if (!pl) return fail(NTT_EINVAL, "plan is NULL");
  if (pl->numeric) return fail(NTT_EUNSUPPORTED, "truncated transforms take integer-word plans");
  if (batch == 0) {
    *done = true;
    return NTT_OK;
  }
  if (!in || !out) return fail(NTT_EINVAL, "NULL vector pointer");
  const size_t esz = pl->wbits / 8;
  if (!aligned_to(in, esz) || !aligned_to(out, esz)) return fail(NTT_EINVAL, "vectors must be %zu-byte aligned", esz);
  if (batch > 0xFFFFFFFFull) return fail(NTT_EINVAL, "batch too large");
  if (!tft_rows_ok(pl))
    return fail(NTT_EUNSUPPORTED, "truncated transforms of length 2^%u: columns of 2^%u words exceed the supported 2^10",
                pl->log2n, pl->L1);
  const size_t need = tft_ws_bytes(pl, batch);
  if (ws_bytes < need || (need && !ws)) return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != pl->device) return fail(NTT_EINVAL, "plan belongs to device %d, current device is %d", pl->device, dev);
  return NTT_OK;
}

// out[i] = a^_[i] (TFT order) for i < l_out, from l_in coefficients (zero above).
int run_tft_forward(const ntt_plan* pl, const void* in, size_t l_in, void* out, size_t l_out, size_t batch,
                    size_t in_stride, size_t out_stride, void* ws, size_t ws_bytes, hipStream_t stream) {
  bool done = false;
  int rc = tft_check(pl, in, out, batch, ws_bytes, ws, &done);
  if (rc || done) return rc ? rc : ok();
  const size_t n = (size_t)1 << pl->log2n;
  if (l_in > n || l_out > n || l_in > in_stride || l_out > out_stride)
    return fail(NTT_EINVAL, "lengths l_in = %zu, l_out = %zu must be <= n = %zu and <= their strides", l_in, l_out, n);
  if (l_out == 0) return ok();
  const int wb = (int)pl->wbits;
  if (pl->passes == 1) {
    LdsNttArgs a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.stride = in_stride;
    a.out_stride = out_stride;
    a.pc = pl->passc;
    a.tw = pl->tw;
    a.twi = pl->twi;
    a.L = pl->log2n;
    a.bitrev = 1;
    a.batch = (uint32_t)batch;
    a.nin = (uint32_t)l_in;
    a.nout = (uint32_t)l_out;
    if (l_in == 0) {  // nothing to read: every value is 0
      for (size_t v = 0; v < batch; ++v)
        HIP_TRY(launch_fill_u32((uint32_t*)((unsigned char*)out + v * out_stride * (wb / 8)), l_out * (wb / 32), 0u, stream));
      return ok();
    }
    HIP_TRY(launch_lds_ntt(wb, false, a, stream));
    return ok();
  }
  const size_t n1 = (size_t)1 << pl->L2;
  const uint32_t lam = (uint32_t)((l_out + n1 - 1) / n1);
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.pc = pl->passc;
  a.tw = pl->tw;
  a.twi = pl->twi;
  a.tlo = pl->tlo;
  a.thi = pl->thi;
  a.batch = (uint32_t)batch;
  a.in = in;
  a.in_stride = in_stride;
  a.valid = l_in;
  a.out = ws;
  a.out_stride = (size_t)lam * n1;
  a.rows = lam;
  HIP_TRY(launch_col_fwd(wb, a, (int)pl->L1, (int)pl->L2, stream));
  a.in = ws;
  a.in_stride = (size_t)lam * n1;
  a.out = out;
  a.out_stride = out_stride;
  a.valid = l_out;
  HIP_TRY(launch_row_fwd(wb, a, (int)pl->L1, (int)pl->L2, stream));
  return ok();
}

// out[0 .. l) = the l coefficients whose TFT values (TFT order) are in[0 .. l).
int run_tft_inverse(const ntt_plan* pl, const void* in, void* out, size_t l, size_t batch, size_t in_stride,
                    size_t out_stride, void* ws, size_t ws_bytes, hipStream_t stream) {
  bool done = false;
  int rc = tft_check(pl, in, out, batch, ws_bytes, ws, &done);
  if (rc || done) return rc ? rc : ok();
  const size_t n = (size_t)1 << pl->log2n;
  if (l > n || l > in_stride || l > out_stride)
    return fail(NTT_EINVAL, "length l = %zu must be <= n = %zu and <= the strides", l, n);
  if (l == 0) return ok();
  const int wb = (int)pl->wbits;
  const size_t esz = wb / 8;
  if (pl->passes == 1) {
    TftArgs a = pl->wbits == 32 ? tft_args<uint32_t>(pl) : tft_args<uint64_t>(pl);
    a.in = in;
    a.out = out;
    a.in_stride = in_stride;
    a.out_stride = out_stride;
    a.valid = l;
    a.lam = (uint32_t)l;
    a.batch = (uint32_t)batch;
    HIP_TRY(launch_vec_itft(wb, a, stream));
    return ok();
  }
  const size_t n1 = (size_t)1 << pl->L2;
  const uint32_t lam = (uint32_t)((l + n1 - 1) / n1);
  const uint32_t lp = (uint32_t)(l - (size_t)(lam - 1) * n1);  // known values of the last row: 1 .. n1
  unsigned char* wsb = (unsigned char*)ws;
  void* W = wsb;  // column-domain values, lam rows per vector
  void* rowbuf = wsb + align256(n * esz * batch);
  const size_t wstride = (size_t)lam * n1;
  const uint32_t full_rows = lp == n1 ? lam : lam - 1;
  // (1) inverse row transforms of the fully known rows, normalized, untwisted
  if (full_rows > 0) {
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.pc = pl->passc;
    a.tw = pl->tw;
    a.twi = pl->twi;
    a.tilo = pl->tilo;
    a.tihi = pl->tihin1;
    a.batch = (uint32_t)batch;
    a.in = in;
    a.in_stride = in_stride;
    a.out = W;
    a.out_stride = wstride;
    a.rows = full_rows;
    HIP_TRY(launch_row_inv(wb, a, (int)pl->L1, (int)pl->L2, false, stream));
  }
  TftArgs t = pl->wbits == 32 ? tft_args<uint32_t>(pl) : tft_args<uint64_t>(pl);
  t.batch = (uint32_t)batch;
  t.rowbuf = rowbuf;
  t.rowbuf_stride = n1;
  if (lp < n1) {
    // (2) columns c >= lp hold lam - 1 unknown inputs: their inverse TFT, and their
    //     value at TFT position lam - 1 (twisted as the row pass twists row lam - 1)
    if (lam > 1) {
      t.in = W;
      t.in_stride = wstride;
      t.out = out;
      t.out_stride = out_stride;
      t.valid = l;
      t.lam = lam - 1;
      t.c_lo = lp;
      t.c_hi = (uint32_t)n1;
      t.eval_next = 1;
      const uint64_t wcol = powmod(pl->g, (pl->p - 1) >> pl->L1, pl->p);  // w_(2^L1)
      const uint64_t z = powmod(wcol, brev(lam - 1, (int)pl->L1), pl->p);
      t.zeta = z;
      t.zeta_s = pl->wbits == 32 ? (uint64_t)(((u128)z << 32) / pl->p) : (uint64_t)(((u128)z << 64) / pl->p);
      HIP_TRY(launch_col_itft(wb, t, stream));
    } else {
      // one row only: the columns above lp are zero, and so is their TFT value
      for (size_t v = 0; v < batch; ++v)
        HIP_TRY(launch_fill_u32((uint32_t*)((unsigned char*)rowbuf + v * n1 * esz), n1 * (esz / 4), 0u, stream));
    }
    // (3) the last row: lp known TFT values, known twisted inputs at c >= lp
    t.eval_next = 0;
    t.in = in;
    t.in_stride = in_stride;
    t.out = W;
    t.out_stride = wstride;
    t.lam = lp;
    t.lastrow = lam - 1;
    HIP_TRY(launch_row_itft(wb, t, stream));
  }
  // (4) columns c < lp (all columns when the last row is full): lam known values each
  t.eval_next = 0;
  t.in = W;
  t.in_stride = wstride;
  t.out = out;
  t.out_stride = out_stride;
  t.valid = l;
  t.lam = lam;
  t.c_lo = 0;
  t.c_hi = lp;
  HIP_TRY(launch_col_itft(wb, t, stream));
  return ok();
}

// ============================================================================ C ABI
extern "C" {

const char* ntt_strerror(int code) {
  switch (code) {
    case NTT_OK: return "success";
    case NTT_EINVAL: return "invalid argument";
    case NTT_ENOTPRIME: return "modulus is not prime";
    case NTT_ENOROOT: return "no root of unity of the requested order";
    case NTT_ERANGE: return "input is not a canonical residue";
    case NTT_ENOMEM: return "out of memory or workspace too small";
    case NTT_EDEVICE: return "device error";
    case NTT_EUNSUPPORTED: return "unsupported modulus or size";
    default: return "unknown error";
  }
}

const char* ntt_last_error(void) { return g_last_error.c_str(); }

int ntt_is_prime(uint64_t n) { return is_prime_u64(n) ? 1 : 0; }

uint64_t ntt_smallest_generator(uint64_t p) { return is_prime_u64(p) ? smallest_generator(p) : 0; }

uint64_t ntt_find_prime(uint32_t bits, uint32_t l) {
  if (bits < 2 || bits > 63 || l >= bits) return 0;
  const uint64_t bound = 1ull << bits;
  for (uint64_t k = (bound - 2) >> l; k > 0; --k) {
    const uint64_t p = (k << l) + 1;
    if (p < bound && is_prime_u64(p)) return p;
  }
  return 0;
}

int ntt_plan_create(ntt_plan** out, uint64_t p, uint64_t g, uint32_t log2n, uint32_t flags, void* hip_stream) {
  (void)hip_stream;
  if (!out) return fail(NTT_EINVAL, "out is NULL");
  *out = nullptr;
  try {
    int rc = create_plan(out, p, g, log2n, flags);
    return rc ? rc : ok();
  } catch (...) {
    return fail(NTT_ENOMEM, "exception during plan creation");
  }
}

int ntt_plan_destroy(ntt_plan* plan) {
  if (!plan) return ok();
  if (plan->dmem) (void)hipFree(plan->dmem);
  delete plan;
  return ok();
}

int ntt_plan_get_info(const ntt_plan* plan, ntt_plan_info* info) {
  if (!plan || !info) return fail(NTT_EINVAL, "NULL argument");
  info->p = plan->p;
  info->g = plan->g;
  info->w = plan->w;
  info->w_inv = plan->winv;
  info->n_inv = plan->ninv;
  info->log2n = plan->log2n;
  info->word_bits = plan->wbits;
  info->flags = plan->flags;
  info->passes = plan->passes;
  info->row_log2 = plan->passes > 1 ? plan->L2 : 0;
  return ok();
}

size_t ntt_workspace_bytes(const ntt_plan* plan, size_t batch) {
  if (!plan || plan->passes == 1) return 0;
  const bool natural_any = !(plan->flags & NTT_BITREV_OUT) || !(plan->flags & NTT_BITREV_IN);
  if (!natural_any) return 0;
  return ((size_t)1 << plan->log2n) * (plan->wbits / 8) * batch;
}

int ntt_forward(const ntt_plan* plan, const void* in, void* out, size_t batch, size_t stride_elems, void* workspace,
                size_t ws_bytes, void* hip_stream) {
  try {
    return run_transform(plan, false, in, out, batch, stride_elems, workspace, ws_bytes, (hipStream_t)hip_stream);
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in ntt_forward");
  }
}

int ntt_inverse(const ntt_plan* plan, const void* in, void* out, size_t batch, size_t stride_elems, void* workspace,
                size_t ws_bytes, void* hip_stream) {
  try {
    return run_transform(plan, true, in, out, batch, stride_elems, workspace, ws_bytes, (hipStream_t)hip_stream);
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in ntt_inverse");
  }
}

size_t ntt_tft_workspace_bytes(const ntt_plan* plan, size_t batch) { return tft_ws_bytes(plan, batch); }

int ntt_tft_forward(const ntt_plan* plan, const void* in, size_t l_in, void* out, size_t l_out, size_t batch,
                    size_t in_stride, size_t out_stride, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    return run_tft_forward(plan, in, l_in, out, l_out, batch, in_stride, out_stride, workspace, ws_bytes,
                           (hipStream_t)hip_stream);
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in ntt_tft_forward");
  }
}

int ntt_tft_inverse(const ntt_plan* plan, const void* in, void* out, size_t l, size_t batch, size_t in_stride,
                    size_t out_stride, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    return run_tft_inverse(plan, in, out, l, batch, in_stride, out_stride, workspace, ws_bytes,
                           (hipStream_t)hip_stream);
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in ntt_tft_inverse");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------- products
namespace {

struct ProductShape {
  uint64_t p;
  int wb;         // word bits
  int L;          // log2 of the transform length
  bool fused;     // one workgroup per product
  size_t lc;
  int split = 0;  // single products: 2^split workgroups (latency path), 0 = not split
};

// Largest log2 N for which a single product (polymul_modp, each prime of intmul_crt)
// takes the fused one-workgroup kernel; above it the two-pass path.  Batches always
// take the fused kernel up to its limit.
// Size class of a fused product (fused_class), except that with the tuning choice
// fused.m15.w32 = 1 32-bit transforms of 2^16 take class 4: two sub-problems of 2^15
// points instead of four of 2^14.
int fclass(int wb, int L) {
  if (wb == 32 && L == 16 && tune_value("fused.m15.w32", 0) != 0) return 4;
  return fused_class(wb, L);
}

int fused_limit(int wb) { return (int)tune_value(tune_key("fused.single.max", wb, -1), fused_max_log2n(wb)); }

// Path of a single product: the split latency path when a split depth is chosen for
// its size, else the fused kernel up to fused_limit, else the two-pass path.
void single_path(ProductShape* s) {
  s->split = (int)tune_value(tune_key("single.split", s->wb, s->L), 0);
  if (s->split && !split_supported(s->wb, s->L, s->split)) s->split = 0;
  s->fused = !s->split && s->L <= fused_limit(s->wb);
}

int shape_of(uint64_t p, size_t la, size_t lb, ProductShape* s) {
  int l = 0;
  int rc = check_modulus(p, &l);
  if (rc) return rc;
  s->p = p;
  s->wb = p < (1ull << 31) ? 32 : 64;
  s->lc = la + lb - 1;
  s->L = ceil_log2(s->lc);
  if (s->L > l)
    return fail(NTT_ENOROOT, "product length %zu needs 2^%d | p - 1 (2-adic order %d)", s->lc, s->L, l);
  if (s->L > 26) return fail(NTT_EUNSUPPORTED, "product length %zu too large", s->lc);
  s->fused = s->L <= fused_max_log2n(s->wb);
  return NTT_OK;
}

size_t multipass_product_ws(const ProductShape& s) { return s.fused ? 0 : 2 * align256(((size_t)1 << s.L) * (s.wb / 8)); }

int current_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  return device_ctx(dev)->cus;
}

// Workspace of one fused launch of `count` products of class `cls`.
size_t fused_launch_ws(int wb, int cls, size_t count, int cus) {
  const size_t words = fused_park_words(wb, cls);
  if (!words || !count) return 0;
  return align256((size_t)fused_grid(wb, cls, count, cus) * words * (wb / 8));
}

size_t single_product_ws(const ProductShape& s, int cus) {
  if (s.split) return align256(((size_t)1 << s.L) * (s.wb / 8));  // the 2^split partials
  return s.fused ? fused_launch_ws(s.wb, fclass(s.wb, s.L), 1, cus) : multipass_product_ws(s);
}

// Two-pass product of one pair (section 5.2 with Algorithm 1): column passes of
// both operands, the fused row pass, and the inverse column pass into c.
int run_multipass_product(const ntt_plan* pl, const void* a, size_t la, const void* b, size_t lb, void* c, size_t lc,
                          bool u16_inputs, void* ws, hipStream_t stream) {
  const int wb = (int)pl->wbits;
  const int wk = pl->numeric ? kWordF64 : wb;  // kernel word code
  const size_t N = (size_t)1 << pl->log2n;
  unsigned char* w = (unsigned char*)ws;
  void* A = w;
  void* B = w + align256(N * (wb / 8));
  PassArgs x;
  memset(&x, 0, sizeof(x));
  x.pc = pl->passc;
  x.tw = pl->tw;
  x.twi = pl->twi;
  x.tlo = pl->tlo;
  x.thi = pl->thi;
  x.tilo = pl->tilo;
  x.tihi = pl->tihi;  // no n^-1: the Montgomery scale folded into b carries it
  x.batch = 1;
  x.in_u16 = u16_inputs ? 1 : 0;
  const int L1 = (int)pl->L1, L2 = (int)pl->L2;
  // Section 5.1's TFT at row granularity: only the first lam = ceil(lc / 2^L2) rows of
  // Algorithm 1's step 3 are needed; the columns are then inverted by the inverse TFT
  // (the product's coefficients at positions >= lc are the known zero inputs).
  const size_t n1 = (size_t)1 << L2;
  const uint32_t lam = (uint32_t)((lc + n1 - 1) / n1);
  // (measured on gfx950: the column inverse TFT costs more than the rows it saves, so
  // this is a tuning choice, off by default)
  const bool trunc = lam < (1u << L1) && !pl->numeric && tft_rows_ok(pl) &&
                     tune_value(tune_key("tft.rows", wb, -1), 0) != 0;
  x.in = a;
  x.out = A;
  x.valid = la;
  x.scale = 0;
  x.rows = trunc ? lam : 0;
  HIP_TRY(launch_col_fwd(wk, x, L1, L2, stream));
  x.in = b;
  x.out = B;
  x.valid = lb;
  x.scale = trunc ? 3 : 1;  // the row inverse normalized by 2^-L2 when the columns take the inverse TFT
  HIP_TRY(launch_col_fwd(wk, x, L1, L2, stream));
  x.in_u16 = 0;
  x.scale = 0;
  x.in = A;
  x.in2 = B;
  x.out = A;
  HIP_TRY(launch_row_polymul(wk, x, L1, L2, stream));
  if (trunc) {
    TftArgs t = wb == 32 ? tft_args<uint32_t>(pl) : tft_args<uint64_t>(pl);
    t.in = A;
    t.in_stride = N;
    t.out = c;
    t.out_stride = N;
    t.valid = lc;
    t.lam = lam;
    t.c_lo = 0;
    t.c_hi = (uint32_t)n1;
    t.batch = 1;
    HIP_TRY(launch_col_itft(wb, t, stream));
    return NTT_OK;
  }
  x.rows = 0;
  x.in = A;
  x.out = c;
  x.valid = lc;
  HIP_TRY(launch_col_inv(wk, x, L1, L2, stream));
  return NTT_OK;
}

// Two-pass products of the same operands modulo n primes of equal transform length
// (several moduli in one launch, section 2.2's Remark 6): the 2n column passes, the n
// fused row passes and the n inverse column passes each share one launch.  input: 0
// canonical residues, 1 16-bit limbs, 2 32-bit words that may exceed the primes.
// Workspace: n * 2 * N words.
int run_multipass_products(ntt_plan* const* pls, int n, const void* a, size_t la, const void* b, size_t lb,
                           void* const* c, size_t lc, int input, void* ws, hipStream_t stream) {
  if (n < 1 || 2 * n > kMaxPassJobs) return fail(NTT_EINVAL, "too many primes in one launch");
  const int wb = (int)pls[0]->wbits;
  const size_t N = (size_t)1 << pls[0]->log2n;
  const int L1 = (int)pls[0]->L1, L2 = (int)pls[0]->L2;
  for (int i = 1; i < n; ++i)
    if ((int)pls[i]->wbits != wb || pls[i]->L1 != (uint32_t)L1 || pls[i]->L2 != (uint32_t)L2)
      return fail(NTT_EINVAL, "products of one launch need the same transform shape");
  unsigned char* w = (unsigned char*)ws;
  const size_t vec = align256(N * (wb / 8));
  PassJobs fwd, row, inv;
  memset(&fwd, 0, sizeof(fwd));
  memset(&row, 0, sizeof(row));
  memset(&inv, 0, sizeof(inv));
  for (int i = 0; i < n; ++i) {
    const ntt_plan* pl = pls[i];
    void* A = w + (size_t)(2 * i) * vec;
    void* B = w + (size_t)(2 * i + 1) * vec;
    PassArgs x;
    memset(&x, 0, sizeof(x));
    x.pc = pl->passc;
    x.tw = pl->tw;
    x.twi = pl->twi;
    x.tlo = pl->tlo;
    x.thi = pl->thi;
    x.tilo = pl->tilo;
    x.tihi = pl->tihi;  // no n^-1: the Montgomery scale folded into b carries it
    x.batch = 1;
    x.in_u16 = input == 1 ? 1 : 0;
    x.in = a;
    x.out = A;
    x.valid = la;
    x.scale = input == 2 ? 2 : 0;
    fwd.j[fwd.n++] = x;
    x.in = b;
    x.out = B;
    x.valid = lb;
    x.scale = 1;
    fwd.j[fwd.n++] = x;
    x.in_u16 = 0;
    x.scale = 0;
    x.in = A;
    x.in2 = B;
    x.out = A;
    row.j[row.n++] = x;
    x.in2 = nullptr;
    x.out = c[i];
    x.valid = lc;
    inv.j[inv.n++] = x;
  }
  HIP_TRY(launch_col_fwd_jobs(wb, fwd, L1, L2, stream));
  HIP_TRY(launch_row_polymul_jobs(wb, row, L1, L2, stream));
  HIP_TRY(launch_col_inv_jobs(wb, inv, L1, L2, stream));
  return NTT_OK;
}

FusedItem fused_item(const ntt_plan* pl, const void* a, size_t la, const void* b, size_t lb, void* c) {
  FusedItem it;
  memset(&it, 0, sizeof(it));
  it.a = a;
  it.b = b;
  it.c = c;
  it.la = la;
  it.lb = lb;
  it.cst = pl->polyc;
  it.tw = pl->tw;
  it.twi = pl->twi;
  it.log2n = pl->log2n;
  return it;
}

// Scratch of a batch beyond its descriptor array: one park area per fused launch that
// parks partials (the launches may run at once, on forked streams), then the largest
// two-pass product (they run one after the other).
size_t batch_scratch(const std::vector<ProductShape>& shapes, int cus, size_t* nfused_out) {
  size_t per_class[2][kFusedClasses] = {};
  size_t nfused = 0, big = 0, parks = 0;
  for (const ProductShape& s : shapes) {
    if (s.L < 0) continue;
    if (s.fused) {
      ++nfused;
      ++per_class[s.wb == 64][fclass(s.wb, s.L)];
    } else {
      big = std::max(big, multipass_product_ws(s));
    }
  }
  for (int w = 0; w < 2; ++w)
    for (int c = 0; c < kFusedClasses; ++c) parks += fused_launch_ws(w ? 64 : 32, c, per_class[w][c], cus);
  if (nfused_out) *nfused_out = nfused;
  return parks + big;
}

// The independent launches of one batch call (one per size class, and the two-pass
// products as one sequence): unit 0 runs on the caller's stream, unit k > 0 on a
// stream forked from it (at most kForkLanes per caller, default priority) and joined
// back into it, so that classes that fill few CUs and the two-pass products overlap.
// Everything stays on the caller's stream while a graph is being captured, for a single
// unit, or with the tuning choice batch.fork = 0.
constexpr int kForkLanes = 8;
constexpr size_t kForkCallers = 8;

class Fork {
 public:
  Fork(hipStream_t s, int units) : main_(s), units_(units) {}
  ~Fork() {
    if (e0_) (void)hipEventDestroy(e0_);
  }
  int begin() {
    if (units_ < 2 || capturing(main_) || tune_value("batch.fork", 1) == 0) return NTT_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceCtx* ctx = device_ctx(dev);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      auto it = ctx->lanes.find(main_);
      if (it == ctx->lanes.end()) {
        DeviceCtx::Lanes moved;
        if (ctx->lanes.size() >= kForkCallers) {  // hand the least recently used caller's lanes over
          auto old = ctx->lanes.begin();
          for (auto j = ctx->lanes.begin(); j != ctx->lanes.end(); ++j)
            if (j->second.used < old->second.used) old = j;
          moved = std::move(old->second);
          ctx->lanes.erase(old);
        }
        it = ctx->lanes.emplace(main_, std::move(moved)).first;
      }
      std::vector<hipStream_t>& v = it->second.s;
      it->second.used = ++ctx->lane_clock;
      const int want = std::min(units_ - 1, kForkLanes);
      while ((int)v.size() < want) {
        hipStream_t t = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));  // default priority
        v.push_back(t);
      }
      lanes_.assign(v.begin(), v.begin() + want);
    }
    HIP_TRY(hipEventCreateWithFlags(&e0_, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(e0_, main_));
    for (hipStream_t l : lanes_) HIP_TRY(hipStreamWaitEvent(l, e0_, 0));
    return NTT_OK;
  }
  // unit k > 0 on lane (k - 1) mod kForkLanes: units beyond the lanes share them in turn
  hipStream_t lane(int k) const { return k == 0 || lanes_.empty() ? main_ : lanes_[(k - 1) % lanes_.size()]; }
  int join() {
    for (hipStream_t l : lanes_) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      const hipError_t r1 = hipEventRecord(e, l);
      const hipError_t r2 = r1 == hipSuccess ? hipStreamWaitEvent(main_, e, 0) : r1;
      (void)hipEventDestroy(e);
      HIP_TRY(r2);
    }
    lanes_.clear();
    return NTT_OK;
  }

 private:
  hipStream_t main_;
  int units_;
  std::vector<hipStream_t> lanes_;
  hipEvent_t e0_ = nullptr;
};

// polymul_modp's checks and launches; create_plans = false: a missing plan is an
// error instead of being created (no device allocation).
int polymul_modp_run(uint64_t p, const void* a, size_t la, const void* b, size_t lb, void* c, void* workspace,
                     size_t ws_bytes, hipStream_t stream, bool create_plans, const char* where) {
  try {
    if (la == 0 || lb == 0) return ok();
    if (!a || !b || !c) return fail(NTT_EINVAL, "NULL operand pointer");
    ProductShape s;
    int rc = shape_of(p, la, lb, &s);
    if (rc) return rc;
    single_path(&s);
    const size_t esz = s.wb / 8;
    if (!aligned_to(a, esz) || !aligned_to(b, esz) || !aligned_to(c, esz))
      return fail(NTT_EINVAL, "operands must be %zu-byte aligned", esz);
    const size_t need = single_product_ws(s, current_cus());
    if (ws_bytes < need || (need && !workspace))
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    ntt_plan* pl = nullptr;
    rc = cached_plan(p, (uint32_t)s.L, &pl, false, true, create_plans);
    if (rc) return rc;
    if (s.split) {
      SplitArgs x;
      memset(&x, 0, sizeof(x));
      x.a = a;
      x.b = b;
      x.c = c;
      x.la = la;
      x.lb = lb;
      x.cst = pl->polyc;
      x.tw = pl->tw;
      x.twi = pl->twi;
      x.park = workspace;
      {
        const size_t S = (size_t)1 << (s.L - s.split);
        x.lam = (uint32_t)std::min<size_t>((size_t)1 << s.split, (s.lc + S - 1) / S);
      }
      HIP_TRY(launch_split(s.wb, x, s.L, s.split, stream));
      return ok();
    }
    if (s.fused) {
      FusedBatch fb;
      memset(&fb, 0, sizeof(fb));
      fb.items = nullptr;
      fb.park = workspace;
      fb.count = 1;
      fb.single = fused_item(pl, a, la, b, lb, c);
      HIP_TRY(launch_fused(s.wb, fclass(s.wb, s.L), fb, 1, stream));
      return ok();
    }
    rc = run_multipass_product(pl, a, la, b, lb, c, s.lc, false, workspace, stream);
    return rc ? rc : ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in %s", where);
  }
}

}  // namespace

extern "C" {

size_t polymul_workspace_bytes(uint64_t p, size_t la, size_t lb) {
  if (la == 0 || lb == 0) return 0;
  ProductShape s;
  if (shape_of(p, la, lb, &s)) return 0;
  single_path(&s);
  return single_product_ws(s, current_cus());
}

int polymul_modp(uint64_t p, const void* a, size_t la, const void* b, size_t lb, void* c, void* workspace,
                 size_t ws_bytes, void* hip_stream) {
  return polymul_modp_run(p, a, la, b, lb, c, workspace, ws_bytes, (hipStream_t)hip_stream, true, "polymul_modp");
}

size_t polymul_batch_workspace_bytes(const ntt_polymul_desc* d, size_t count) {
  if (!d && count) return 0;
  std::vector<ProductShape> shapes(count);
  for (size_t i = 0; i < count; ++i) {
    shapes[i].L = -1;
    if (d[i].la == 0 || d[i].lb == 0) continue;
    if (shape_of(d[i].p, d[i].la, d[i].lb, &shapes[i])) shapes[i].L = -1;
  }
  size_t nfused = 0;
  const size_t scratch = batch_scratch(shapes, current_cus(), &nfused);
  return align256(nfused * sizeof(FusedItem)) + scratch;
}

int polymul_modp_batch(const ntt_polymul_desc* d, size_t count, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    if (capturing(stream))
      return fail(NTT_EINVAL, "polymul_modp_batch copies host descriptors and cannot be captured in a graph: "
                  "use a polymul_batch_create handle");
    if (count == 0) return ok();
    if (!d) return fail(NTT_EINVAL, "descriptor array is NULL");
    std::vector<ProductShape> shapes(count);
    size_t nfused = 0;
    for (size_t i = 0; i < count; ++i) {
      if (d[i].la == 0 || d[i].lb == 0) {
        shapes[i].L = -1;
        continue;
      }
      if (!d[i].a || !d[i].b || !d[i].c) return fail(NTT_EINVAL, "descriptor %zu: NULL operand pointer", i);
      int rc = shape_of(d[i].p, d[i].la, d[i].lb, &shapes[i]);
      if (rc) {
        std::string m = g_last_error;
        return fail(rc, "descriptor %zu: %s", i, m.c_str());
      }
      const size_t esz = shapes[i].wb / 8;
      if (!aligned_to(d[i].a, esz) || !aligned_to(d[i].b, esz) || !aligned_to(d[i].c, esz))
        return fail(NTT_EINVAL, "descriptor %zu: operands must be %zu-byte aligned", i, esz);
    }
    const int cus = current_cus();
    const size_t scratch = batch_scratch(shapes, cus, &nfused);
    const size_t need = align256(nfused * sizeof(FusedItem)) + scratch;
    if (ws_bytes < need || (need && !workspace))
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceCtx* ctx = device_ctx(dev);
    // Group the fused items by (word size, size class), in one contiguous upload.
    std::vector<FusedItem> items;
    items.reserve(nfused);
    struct Group { int wb, cls; size_t first, count; };
    std::vector<Group> groups;
    for (int wb : {32, 64}) {
      for (int cls = 0; cls < kFusedClasses; ++cls) {
        const size_t first = items.size();
        for (size_t i = 0; i < count; ++i) {
          const ProductShape& s = shapes[i];
          if (s.L < 0 || !s.fused || s.wb != wb || fclass(wb, s.L) != cls) continue;
          ntt_plan* pl = nullptr;
          int rc = cached_plan(s.p, (uint32_t)s.L, &pl);
          if (rc) return rc;
          items.push_back(fused_item(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c));
        }
        if (items.size() > first) groups.push_back({wb, cls, first, items.size() - first});
      }
    }
    FusedItem* ditems = (FusedItem*)workspace;
    if (!items.empty()) {
      int rc = upload(ctx, ditems, items.data(), items.size() * sizeof(FusedItem), stream);
      if (rc) return rc;
    }
    unsigned char* ws = (unsigned char*)workspace + align256(nfused * sizeof(FusedItem));
    const bool any_big = nfused < count && std::any_of(shapes.begin(), shapes.end(),
                                                       [](const ProductShape& s) { return s.L >= 0 && !s.fused; });
    // unit 0 (the caller's stream): the multi-pass sequence, the longest; then the groups
    const int g0 = any_big ? 1 : 0;
    Fork fork(stream, (int)groups.size() + g0);
    int rc = fork.begin();
    if (rc) return rc;
    for (size_t k = 0; k < groups.size(); ++k) {
      const Group& g = groups[k];
      FusedBatch fb;
      memset(&fb, 0, sizeof(fb));
      fb.items = ditems + g.first;
      fb.park = ws;  // this launch's own park area
      fb.count = (int)g.count;
      HIP_TRY(launch_fused(g.wb, g.cls, fb, fused_grid(g.wb, g.cls, g.count, cus), fork.lane((int)k + g0)));
      ws += fused_launch_ws(g.wb, g.cls, g.count, cus);
    }
    for (size_t i = 0; i < count; ++i) {
      const ProductShape& s = shapes[i];
      if (s.L < 0 || s.fused) continue;
      ntt_plan* pl = nullptr;
      rc = cached_plan(s.p, (uint32_t)s.L, &pl);
      if (rc) return rc;
      rc = run_multipass_product(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c, s.lc, false, ws, fork.lane(0));
      if (rc) return rc;
    }
    rc = fork.join();
    if (rc) return rc;
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in polymul_modp_batch");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------- reusable batches
constexpr int kF64Group = -64;      // group word size of residues held in doubles, p < 2^49
constexpr int kF64BandGroup = -65;  // the same with 2^49 <= p < 2^50 (the kernels' band variant)
struct ntt_batch {
  int device;
  void* ditems;  // device FusedItem array (owned)
  struct Group { int wb, cls; size_t first, count; };
  std::vector<Group> groups;
  struct Big { const ntt_plan* pl; const void *a, *b; void* c; size_t la, lb, lc; };
  std::vector<Big> big;
  size_t big_ws;  // scratch of a launch: park areas and two-pass products
  int cus;
};

extern "C" {

int polymul_batch_create(ntt_batch** out, const ntt_polymul_desc* d, size_t count) {
  try {
    if (!out) return fail(NTT_EINVAL, "out is NULL");
    *out = nullptr;
    if (g_capturing) return fail(NTT_EINVAL, "polymul_batch_create allocates and cannot run during a graph capture");
    if (count && !d) return fail(NTT_EINVAL, "descriptor array is NULL");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<ProductShape> shapes(count);
    for (size_t i = 0; i < count; ++i) {
      if (d[i].la == 0 || d[i].lb == 0) {
        shapes[i].L = -1;
        continue;
      }
      if (!d[i].a || !d[i].b || !d[i].c) return fail(NTT_EINVAL, "descriptor %zu: NULL operand pointer", i);
      int rc = shape_of(d[i].p, d[i].la, d[i].lb, &shapes[i]);
      if (rc) {
        std::string m = g_last_error;
        return fail(rc, "descriptor %zu: %s", i, m.c_str());
      }
      const size_t esz = shapes[i].wb / 8;
      if (!aligned_to(d[i].a, esz) || !aligned_to(d[i].b, esz) || !aligned_to(d[i].c, esz))
        return fail(NTT_EINVAL, "descriptor %zu: operands must be %zu-byte aligned", i, esz);
    }
    ntt_batch* bt = new ntt_batch();
    bt->device = dev;
    bt->ditems = nullptr;
    bt->big_ws = 0;
    std::vector<FusedItem> items;
    for (int wb : {32, 64}) {
      for (int cls = 0; cls < kFusedClasses; ++cls) {
        const size_t first = items.size();
        for (size_t i = 0; i < count; ++i) {
          const ProductShape& s = shapes[i];
          if (s.L < 0 || !s.fused || s.wb != wb || fclass(wb, s.L) != cls) continue;
          ntt_plan* pl = nullptr;
          int rc = cached_plan(s.p, (uint32_t)s.L, &pl);
          if (rc) {
            delete bt;
            return rc;
          }
          items.push_back(fused_item(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c));
        }
        if (items.size() > first) bt->groups.push_back({wb, cls, first, items.size() - first});
      }
    }
    for (size_t i = 0; i < count; ++i) {
      const ProductShape& s = shapes[i];
      if (s.L < 0 || s.fused) continue;
      ntt_plan* pl = nullptr;
      int rc = cached_plan(s.p, (uint32_t)s.L, &pl);
      if (rc) {
        delete bt;
        return rc;
      }
      bt->big.push_back({pl, d[i].a, d[i].b, d[i].c, d[i].la, d[i].lb, s.lc});
    }
    bt->cus = current_cus();
    bt->big_ws = batch_scratch(shapes, bt->cus, nullptr);
    if (!items.empty()) {
      if (hipMalloc(&bt->ditems, items.size() * sizeof(FusedItem)) != hipSuccess) {
        delete bt;
        return fail(NTT_ENOMEM, "hipMalloc of batch descriptors failed");
      }
      if (hipMemcpy(bt->ditems, items.data(), items.size() * sizeof(FusedItem), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(bt->ditems);
        delete bt;
        return fail(NTT_EDEVICE, "upload of batch descriptors failed");
      }
    }
    *out = bt;
    return ok();
  } catch (...) {
    return fail(NTT_ENOMEM, "exception in polymul_batch_create");
  }
}

size_t polymul_batch_launch_workspace_bytes(const ntt_batch* batch) { return batch ? batch->big_ws : 0; }

int polymul_batch_launch(const ntt_batch* bt, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    if (!bt) return fail(NTT_EINVAL, "batch is NULL");
    hipStream_t stream = (hipStream_t)hip_stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != bt->device) return fail(NTT_EINVAL, "batch belongs to device %d, current device is %d", bt->device, dev);
    if (ws_bytes < bt->big_ws || (bt->big_ws && !workspace))
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", bt->big_ws, ws_bytes);
    unsigned char* ws = (unsigned char*)workspace;
    // unit 0 (the caller's stream): the multi-pass sequence, the longest; then the groups
    const int g0 = bt->big.empty() ? 0 : 1;
    Fork fork(stream, (int)bt->groups.size() + g0);
    int rc = fork.begin();
    if (rc) return rc;
    for (size_t k = 0; k < bt->groups.size(); ++k) {
      const auto& g = bt->groups[k];
      const hipStream_t st = fork.lane((int)k + g0);
      FusedBatch fb;
      memset(&fb, 0, sizeof(fb));
      fb.items = (const FusedItem*)bt->ditems + g.first;
      fb.park = ws;  // this launch's own park area
      fb.count = (int)g.count;
      if (g.wb == kF64Group || g.wb == kF64BandGroup) {
        HIP_TRY(launch_fused_f64(g.cls, g.wb == kF64BandGroup, fb, fused_grid(64, g.cls, g.count, bt->cus), st));
      } else {
        HIP_TRY(launch_fused(g.wb, g.cls, fb, fused_grid(g.wb, g.cls, g.count, bt->cus), st));
        ws += fused_launch_ws(g.wb, g.cls, g.count, bt->cus);
      }
    }
    for (const auto& b : bt->big) {
      rc = run_multipass_product(b.pl, b.a, b.la, b.b, b.lb, b.c, b.lc, false, ws, fork.lane(0));
      if (rc) return rc;
    }
    rc = fork.join();
    if (rc) return rc;
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in polymul_batch_launch");
  }
}

int polymul_batch_destroy(ntt_batch* bt) {
  if (!bt) return ok();
  if (bt->ditems) (void)hipFree(bt->ditems);
  delete bt;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------- tuning
extern "C" {

int ntt_tune_set(const char* key, int64_t value) {
  if (!key) return fail(NTT_EINVAL, "key is NULL");
  if (!tune_valid(key, value)) return fail(NTT_EINVAL, "unknown tuning key or value out of range: %s = %lld", key,
                                           (long long)value);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = value;
  return ok();
}

int ntt_tune_get(const char* key, int64_t* value) {
  if (!key || !value) return fail(NTT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return fail(NTT_EINVAL, "tuning key %s is not set", key);
  *value = it->second;
  return ok();
}

int ntt_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return ok();
}

int ntt_tune_load(const char* path) {
  if (!path) return fail(NTT_EINVAL, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(NTT_EINVAL, "cannot open %s", path);
  char line[256];
  int lineno = 0;
  std::vector<std::pair<std::string, int64_t>> kv;
  while (fgets(line, sizeof(line), f)) {
    ++lineno;
    char* hash = strchr(line, '#');
    if (hash) *hash = 0;
    char key[128];
    long long v = 0;
    char extra[8];
    const int n = sscanf(line, "%127s %lld %7s", key, &v, extra);
    if (n <= 0) continue;
    if (n != 2 || !tune_valid(key, v)) {
      fclose(f);
      return fail(NTT_EINVAL, "%s:%d: not a valid 'key value' tuning line", path, lineno);
    }
    kv.emplace_back(key, (int64_t)v);
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : kv) g_tune[e.first] = e.second;
  return ok();
}

int ntt_plan_cache_clear(void) {
  if (g_capturing) return fail(NTT_EINVAL, "cannot clear plans during a graph capture");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceCtx* c = device_ctx(dev);
  std::lock_guard<std::mutex> lk(c->mu);
  for (auto& e : c->plans) ntt_plan_destroy(e.second);
  c->plans.clear();
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------- graphs
struct ntt_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

extern "C" {

int ntt_graph_begin(void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  if (!s) return fail(NTT_EINVAL, "graph capture needs a created stream, not the null stream");
  if (g_capturing) return fail(NTT_EINVAL, "a capture is already open on this thread");
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  g_capturing = true;
  return ok();
}

int ntt_graph_end(void* hip_stream, ntt_graph** out) {
  if (!out) return fail(NTT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!g_capturing) return fail(NTT_EINVAL, "no capture is open on this thread");
  g_capturing = false;
  hipStream_t s = (hipStream_t)hip_stream;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || !g) return fail(NTT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(NTT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  ntt_graph* G = new ntt_graph();
  G->graph = g;
  G->exec = x;
  (void)hipGetDevice(&G->device);
  *out = G;
  return ok();
}

int ntt_graph_launch(const ntt_graph* g, void* hip_stream) {
  if (!g) return fail(NTT_EINVAL, "graph is NULL");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->device) return fail(NTT_EINVAL, "graph belongs to device %d, current device is %d", g->device, dev);
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
  return ok();
}

int ntt_graph_destroy(ntt_graph* g) {
  if (!g) return ok();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------- integer product
namespace {

const uint32_t kIntPrimes[3] = {998244353u, 469762049u, 167772161u};
const size_t kIntMaxCoeffs = (size_t)1 << 23;

struct IntLayout {
  size_t lc, npos, N, nblk;
  int L;
  bool fused;
  size_t o_r[3], o_t, o_blk, o_a32, o_b32, o_big, total;
};

IntLayout int_layout(size_t na, size_t nb) {
  IntLayout z;
  memset(&z, 0, sizeof(z));
  z.lc = na + nb - 1;
  z.L = ceil_log2(z.lc);
  z.N = (size_t)1 << z.L;
  z.npos = (na + nb + 1) & ~(size_t)1;
  z.nblk = (z.npos + crt_block_positions() - 1) / crt_block_positions();
  z.fused = z.L <= fused_limit(32);
  size_t off = 0;
  for (int i = 0; i < 3; ++i) {
    z.o_r[i] = off;
    off += align256(z.lc * 4);
  }
  z.o_t = off;
  off += align256(z.nblk * crt_block_positions() * 4);
  z.o_blk = off;
  off += align256(z.nblk * 4);
  if (z.fused) {
    z.o_a32 = off;
    off += align256(na * 4);
    z.o_b32 = off;
    off += align256(nb * 4);
    z.o_big = off;  // park area of the fused launches
    off += fused_launch_ws(32, fclass(32, z.L), 1, current_cus());
  } else {
    z.o_big = off;
    off += 3 * 2 * align256(z.N * 4);  // the three primes' products share their launches
  }
  z.total = off;
  return z;
}

}  // namespace

extern "C" {

size_t intmul_workspace_bytes(size_t na, size_t nb) {
  if (na == 0 || nb == 0) return 0;
  if (na + nb - 1 > kIntMaxCoeffs) return 0;
  return int_layout(na, nb).total;
}

int intmul_crt(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint32_t* c, void* workspace,
               size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    const size_t nc32 = (na + nb + 1) / 2;
    if (nc32 && !c) return fail(NTT_EINVAL, "output pointer is NULL");
    if (!aligned_to(c, 4) || !aligned_to(a, 2) || !aligned_to(b, 2)) return fail(NTT_EINVAL, "misaligned pointer");
    if (na == 0 || nb == 0) {
      HIP_TRY(launch_fill_u32(c, nc32, 0u, stream));
      return ok();
    }
    if (!a || !b) return fail(NTT_EINVAL, "NULL operand pointer");
    if (na + nb - 1 > kIntMaxCoeffs)
      return fail(NTT_EINVAL, "na + nb - 1 = %zu exceeds 2^23 coefficients", na + nb - 1);
    const IntLayout z = int_layout(na, nb);
    if (ws_bytes < z.total || !workspace)
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", z.total, ws_bytes);
    unsigned char* w = (unsigned char*)workspace;
    uint32_t* r[3];
    for (int i = 0; i < 3; ++i) r[i] = (uint32_t*)(w + z.o_r[i]);
    const void* a_in = a;
    const void* b_in = b;
    if (z.fused) {
      uint32_t* a32 = (uint32_t*)(w + z.o_a32);
      uint32_t* b32 = (uint32_t*)(w + z.o_b32);
      HIP_TRY(launch_widen_u16(a, a32, na, stream));
      HIP_TRY(launch_widen_u16(b, b32, nb, stream));
      a_in = a32;
      b_in = b32;
    }
    ntt_plan* pls[3];
    for (int i = 0; i < 3; ++i) {
      int rc = cached_plan(kIntPrimes[i], (uint32_t)z.L, &pls[i]);
      if (rc) return rc;
    }
    if (z.fused) {
      for (int i = 0; i < 3; ++i) {
        FusedBatch fb;
        memset(&fb, 0, sizeof(fb));
        fb.count = 1;
        fb.park = w + z.o_big;
        fb.single = fused_item(pls[i], a_in, na, b_in, nb, r[i]);
        HIP_TRY(launch_fused(32, fclass(32, z.L), fb, 1, stream));
      }
    } else {
      void* outs[3] = {r[0], r[1], r[2]};
      int rc = run_multipass_products(pls, 3, a, na, b, nb, outs, z.lc, 1, w + z.o_big, stream);
      if (rc) return rc;
    }
    CrtArgs x;
    memset(&x, 0, sizeof(x));
    x.r1 = r[0];
    x.r2 = r[1];
    x.r3 = r[2];
    x.lc = z.lc;
    x.npos = z.npos;
    x.t = (uint32_t*)(w + z.o_t);
    x.blk = (uint32_t*)(w + z.o_blk);
    x.c = c;
    const uint64_t p1 = kIntPrimes[0], p2 = kIntPrimes[1], p3 = kIntPrimes[2];
    x.p1 = (uint32_t)p1;
    x.p2 = (uint32_t)p2;
    x.p3 = (uint32_t)p3;
    const uint64_t c12 = invmod(p1 % p2, p2);
    const uint64_t c123 = invmod(mulmod(p1 % p3, p2 % p3, p3), p3);
    x.c12 = (uint32_t)c12;
    x.c12s = (uint32_t)((c12 << 32) / p2);
    x.c123 = (uint32_t)c123;
    x.c123s = (uint32_t)((c123 << 32) / p3);
    x.p1m3 = (uint32_t)(p1 % p3);
    x.p1m3s = (uint32_t)(((p1 % p3) << 32) / p3);
    x.p1p2 = p1 * p2;
    HIP_TRY(launch_crt_carry(x, stream));
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in intmul_crt");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------- integer product, 32-bit chunks
namespace {

// p1 p2 p3 of the three primes (a bit over 2^86).
u128 int_prime_product() { return (u128)kIntPrimes[0] * kIntPrimes[1] * kIntPrimes[2]; }

// Garner constants of the three primes (p1^-1 mod p2, (p1 p2)^-1 mod p3, p1 mod p3,
// with their Function 8 companions) for the 32-bit-chunk tail.
void crt_constants(CrtArgs* x) {
  const uint64_t p1 = kIntPrimes[0], p2 = kIntPrimes[1], p3 = kIntPrimes[2];
  x->p1 = (uint32_t)p1;
  x->p2 = (uint32_t)p2;
  x->p3 = (uint32_t)p3;
  const uint64_t c12 = invmod(p1 % p2, p2);
  const uint64_t c123 = invmod(mulmod(p1 % p3, p2 % p3, p3), p3);
  x->c12 = (uint32_t)c12;
  x->c12s = (uint32_t)((c12 << 32) / p2);
  x->c123 = (uint32_t)c123;
  x->c123s = (uint32_t)((c123 << 32) / p3);
  x->p1m3 = (uint32_t)(p1 % p3);
  x->p1m3s = (uint32_t)(((p1 % p3) << 32) / p3);
  x->p1p2 = p1 * p2;
}

struct Int32Layout {
  size_t lc, npos, N, nblk;
  int L;
  bool fused;
  size_t o_r[3], o_t, o_blk, o_a, o_b, o_big, total;
};

Int32Layout int32_layout(size_t na, size_t nb) {
  Int32Layout z;
  memset(&z, 0, sizeof(z));
  z.lc = na + nb - 1;
  z.L = ceil_log2(z.lc);
  z.N = (size_t)1 << z.L;
  z.npos = na + nb;
  z.nblk = (z.npos + crt_block_positions() - 1) / crt_block_positions();
  z.fused = z.L <= fused_limit(32);
  size_t off = 0;
  for (int i = 0; i < 3; ++i) {
    z.o_r[i] = off;
    off += align256(z.lc * 4);
  }
  z.o_t = off;
  off += align256(z.nblk * crt_block_positions() * 8);
  z.o_blk = off;
  off += align256(z.nblk * 4);
  z.o_a = off;
  off += align256(na * 4);
  z.o_b = off;
  off += align256(nb * 4);
  z.o_big = off;
  off += z.fused ? fused_launch_ws(32, fclass(32, z.L), 1, current_cus()) : 3 * 2 * align256(z.N * 4);
  z.total = off;
  return z;
}

// The product of two na- and nb-chunk integers has coefficients below
// min(na, nb) (2^32 - 1)^2, which the three primes must exceed.
bool int32_fits(size_t na, size_t nb) {
  const u128 m = (u128)std::min(na, nb);
  const u128 cmax = m * (u128)0xFFFFFFFFull * (u128)0xFFFFFFFFull;
  return cmax < int_prime_product() && na + nb - 1 <= kIntMaxCoeffs;
}

}  // namespace

extern "C" {

int intmul_chunk_bits(size_t na16, size_t nb16) {
  // Section 5.3: the largest chunk size h (here 32 or 16) such that
  // H = 2 h + ceil(log2(d + 1)) bits, d the chunk count, stay below p1 p2 p3, and the
  // product's d_a + d_b - 1 coefficients fit the primes' transform lengths.
  if (na16 == 0 || nb16 == 0) return 16;
  for (int h : {32, 16}) {
    const size_t per = (size_t)h / 16;
    const size_t da = (na16 + per - 1) / per, db = (nb16 + per - 1) / per;
    const size_t d = std::max(da, db);
    const int H = 2 * h + ceil_log2(d + 1);
    if (H < 127 && ((u128)1 << H) < int_prime_product() && da + db - 1 <= kIntMaxCoeffs) return h;
  }
  return 0;
}

size_t intmul32_workspace_bytes(size_t na, size_t nb) {
  if (na == 0 || nb == 0) return 0;
  if (!int32_fits(na, nb)) return 0;
  return int32_layout(na, nb).total;
}

int intmul_crt32(const uint32_t* a, size_t na, const uint32_t* b, size_t nb, uint32_t* c, void* workspace,
                 size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    const size_t nc = na + nb;
    if (nc && !c) return fail(NTT_EINVAL, "output pointer is NULL");
    if (!aligned_to(c, 4) || !aligned_to(a, 4) || !aligned_to(b, 4)) return fail(NTT_EINVAL, "misaligned pointer");
    if (na == 0 || nb == 0) {
      HIP_TRY(launch_fill_u32(c, nc, 0u, stream));
      return ok();
    }
    if (!a || !b) return fail(NTT_EINVAL, "NULL operand pointer");
    if (!int32_fits(na, nb))
      return fail(NTT_EINVAL, "%zu x %zu chunks of 32 bits: coefficients could reach p1 p2 p3 or exceed 2^23 of them",
                  na, nb);
    const Int32Layout z = int32_layout(na, nb);
    if (ws_bytes < z.total || !workspace)
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", z.total, ws_bytes);
    unsigned char* w = (unsigned char*)workspace;
    uint32_t* r[3];
    for (int i = 0; i < 3; ++i) r[i] = (uint32_t*)(w + z.o_r[i]);
    uint32_t* ar = (uint32_t*)(w + z.o_a);
    uint32_t* br = (uint32_t*)(w + z.o_b);
    ntt_plan* pls[3];
    for (int i = 0; i < 3; ++i) {
      int rc = cached_plan(kIntPrimes[i], (uint32_t)z.L, &pls[i]);
      if (rc) return rc;
    }
    if (z.fused) {
      for (int i = 0; i < 3; ++i) {
        // chunks of 32 bits exceed the primes: reduce them first
        HIP_TRY(launch_reduce_mod(a, ar, na, kIntPrimes[i], stream));
        HIP_TRY(launch_reduce_mod(b, br, nb, kIntPrimes[i], stream));
        FusedBatch fb;
        memset(&fb, 0, sizeof(fb));
        fb.count = 1;
        fb.park = w + z.o_big;
        fb.single = fused_item(pls[i], ar, na, br, nb, r[i]);
        HIP_TRY(launch_fused(32, fclass(32, z.L), fb, 1, stream));
      }
    } else {
      // the column pass reduces the chunks as it loads them (input kind 2)
      void* outs[3] = {r[0], r[1], r[2]};
      int rc = run_multipass_products(pls, 3, a, na, b, nb, outs, z.lc, 2, w + z.o_big, stream);
      if (rc) return rc;
    }
    CrtArgs x;
    memset(&x, 0, sizeof(x));
    crt_constants(&x);
    x.r1 = r[0];
    x.r2 = r[1];
    x.r3 = r[2];
    x.lc = z.lc;
    x.npos = z.npos;
    x.t = (uint32_t*)(w + z.o_t);
    x.blk = (uint32_t*)(w + z.o_blk);
    x.c = c;
    HIP_TRY(launch_crt32_carry(x, stream));
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in intmul_crt32");
  }
}

}  // extern "C"

// ============================================================================ polynomial matrices
namespace {

// Transform length of the polynomial matrix product: N = 2^L >= 2d - 1.
int polymat_log2(size_t d) {
  const size_t lc = 2 * d - 1;
  int L = 0;
  while (((size_t)1 << L) < lc) ++L;
  return L;
}

int polymat_check(uint64_t p, size_t n, size_t d) {
  if (n == 0 || d == 0) return NTT_OK;
  if (p < 3 || !is_prime_u64(p)) return fail(NTT_ENOTPRIME, "%llu is not an odd prime", (unsigned long long)p);
  if (p >= (1ull << 31)) return fail(NTT_EUNSUPPORTED, "the matrix product takes primes below 2^31");
  if (n > kMatMaxN) return fail(NTT_EUNSUPPORTED, "n = %zu exceeds %u", n, kMatMaxN);
  if (d > ((size_t)1 << 25)) return fail(NTT_EINVAL, "degree bound d = %zu too large", d);
  const int L = polymat_log2(d);
  if (((p - 1) & (((uint64_t)1 << L) - 1)) != 0)
    return fail(NTT_ENOROOT, "2^%d does not divide p - 1 = %llu", L, (unsigned long long)(p - 1));
  return NTT_OK;
}

}  // namespace

extern "C" {

size_t polymatmul_workspace_bytes(uint64_t p, size_t n, size_t d) {
  if (n == 0 || d == 0 || polymat_check(p, n, d)) return 0;
  const size_t N = (size_t)1 << polymat_log2(d);
  return 2 * align256(n * n * N * sizeof(uint32_t));
}

}  // extern "C"

namespace {

// The polynomial matrix product after its argument checks; reduce: the entries of A
// and B are any 32-bit words, reduced modulo p as the first pass loads them.
int polymat_run(uint64_t p, size_t n, const void* A, const void* B, size_t d, void* C, void* workspace,
                hipStream_t stream, bool reduce) {
  {
    const int L = polymat_log2(d);
    const size_t N = (size_t)1 << L, lc = 2 * d - 1, n2 = n * n;
    ntt_plan* pl = nullptr;
    // plain transform passes (no fused row product): the transform-tuned row length
    int rc = cached_plan(p, (uint32_t)L, &pl, false, false);
    if (rc) return rc;
    uint32_t* Ah = (uint32_t*)workspace;
    uint32_t* Bh = (uint32_t*)((unsigned char*)workspace + align256(n2 * N * sizeof(uint32_t)));
    const bool two_pass = pl->passes > 1;
    // forward transforms of the 2 n^2 entries, zero-padded from d to N, TFT order
    PassArgs x;
    memset(&x, 0, sizeof(x));
    if (two_pass) {
      x.pc = pl->passc;
      x.tw = pl->tw;
      x.twi = pl->twi;
      x.tlo = pl->tlo;
      x.thi = pl->thi;
      x.tilo = pl->tilo;
      x.tihi = pl->tihi;  // no 1/N in the inverse: K carries it
      x.batch = (uint32_t)n2;
      x.in_stride = d;
      x.out_stride = N;
      x.valid = d;
      x.scale = reduce ? 2 : 0;
      PassJobs fwd;
      memset(&fwd, 0, sizeof(fwd));
      x.in = A;
      x.out = Ah;
      fwd.j[fwd.n++] = x;
      x.in = B;
      x.out = Bh;
      fwd.j[fwd.n++] = x;
      HIP_TRY(launch_col_fwd_jobs(32, fwd, (int)pl->L1, (int)pl->L2, stream));
      PassArgs r = x;
      r.scale = 0;
      r.in_stride = N;
      r.valid = N;
      PassJobs rows;  // the row passes of A and B as the two jobs of one launch
      memset(&rows, 0, sizeof(rows));
      r.in = Ah;
      r.out = Ah;
      rows.j[rows.n++] = r;
      r.in = Bh;
      r.out = Bh;
      rows.j[rows.n++] = r;
      HIP_TRY(launch_row_fwd_jobs(32, rows, (int)pl->L1, (int)pl->L2, stream));
    } else {
      const uint32_t rp = reduce ? (uint32_t)p : 0u;
      HIP_TRY(launch_copy_rows(Ah, N, N, (const uint32_t*)A, d, d, (uint32_t)n2, stream, rp));
      HIP_TRY(launch_copy_rows(Bh, N, N, (const uint32_t*)B, d, d, (uint32_t)n2, stream, rp));
      LdsNttArgs t;
      memset(&t, 0, sizeof(t));
      t.in = Ah;
      t.out = Ah;
      t.stride = N;
      t.pc = pl->passc;
      t.tw = pl->tw;
      t.twi = pl->twi;
      t.L = (uint32_t)L;
      t.bitrev = 1;
      t.batch = (uint32_t)n2;
      HIP_TRY(launch_lds_ntt(32, false, t, stream));
      t.in = Bh;
      t.out = Bh;
      HIP_TRY(launch_lds_ntt(32, false, t, stream));
    }
    // n x n products at every frequency, written over A's transforms
    MatArgs m;
    memset(&m, 0, sizeof(m));
    m.A = Ah;
    m.B = Bh;
    m.C = Ah;
    m.N = N;
    m.n = (uint32_t)n;
    m.kb = freq_matmul_block((uint32_t)n, N);
    m.p = (uint32_t)p;
    uint32_t inv = (uint32_t)p;  // p^-1 mod 2^32 by Newton's iteration
    for (int i = 0; i < 5; ++i) inv *= 2u - (uint32_t)p * inv;
    m.pinv = inv;
    const uint64_t r32 = (1ull << 32) % p;
    m.r32 = (uint32_t)r32;
    const u128 room = ((u128)1 << 64) - 1 - ((u128)p << 32);
    const u128 fold = room / ((u128)(p - 1) * (p - 1));
    m.fold = (uint32_t)std::min<u128>(fold, (u128)n);
    const uint64_t K = two_pass ? mulmod(r32, pl->ninv, p) : r32;
    m.kw = (uint32_t)K;
    m.kws = (uint32_t)((K << 32) / p);
    HIP_TRY(launch_freq_matmul(m, stream));
    // inverse transforms of C's n^2 entries, the first 2d - 1 coefficients kept
    if (two_pass) {
      PassArgs v = x;
      v.scale = 0;
      v.in = Ah;
      v.in_stride = N;
      v.out = Ah;
      v.out_stride = N;
      v.valid = N;
      HIP_TRY(launch_row_inv(32, v, (int)pl->L1, (int)pl->L2, false, stream));
      v.out = C;
      v.out_stride = lc;
      v.valid = lc;
      HIP_TRY(launch_col_inv(32, v, (int)pl->L1, (int)pl->L2, stream));
    } else {
      LdsNttArgs t;
      memset(&t, 0, sizeof(t));
      t.in = Ah;
      t.out = Ah;
      t.stride = N;
      t.pc = pl->passc;
      t.tw = pl->tw;
      t.twi = pl->twi;
      t.L = (uint32_t)L;
      t.bitrev = 1;
      t.batch = (uint32_t)n2;
      HIP_TRY(launch_lds_ntt(32, true, t, stream));
      HIP_TRY(launch_copy_rows((uint32_t*)C, lc, lc, Ah, N, lc, (uint32_t)n2, stream));
    }
    return NTT_OK;
  }
}

}  // namespace

extern "C" {

int polymatmul_modp(uint64_t p, size_t n, const void* A, const void* B, size_t d, void* C, void* workspace,
                    size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    if (n == 0 || d == 0) return ok();
    if (!A || !B || !C) return fail(NTT_EINVAL, "NULL matrix pointer");
    if (!aligned_to(A, 4) || !aligned_to(B, 4) || !aligned_to(C, 4)) return fail(NTT_EINVAL, "misaligned pointer");
    int rc = polymat_check(p, n, d);
    if (rc) return rc;
    const size_t need = polymatmul_workspace_bytes(p, n, d);
    if (ws_bytes < need || !workspace) return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    rc = polymat_run(p, n, A, B, d, C, workspace, stream, false);
    return rc ? rc : ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in polymatmul_modp");
  }
}

}  // extern "C"

// ============================================================================ integer matrices
namespace {

struct IntMatLayout {
  size_t lc, npos, nblk, o_r[3], o_pm, o_t, o_blk, total;
};

// n x n matrices of na-chunk integers: coefficients of C's entries are sums of n
// products of two chunk polynomials, below n na (2^32 - 1)^2 < p1 p2 p3.
bool intmat_fits(size_t n, size_t na) {
  if (n == 0 || n > kMatMaxN || na == 0 || 2 * na - 1 > ((size_t)1 << 23)) return false;
  const u128 P = (u128)kIntPrimes[0] * kIntPrimes[1] * kIntPrimes[2];
  const u128 m = (u128)0xFFFFFFFFull * 0xFFFFFFFFull;
  return (u128)n * na <= P / m && (u128)n * na * m < P;
}

IntMatLayout intmat_layout(size_t n, size_t na) {
  IntMatLayout z;
  memset(&z, 0, sizeof(z));
  const size_t n2 = n * n;
  z.lc = 2 * na - 1;
  z.npos = 2 * na + 1;  // a sum of n products can carry one limb past 2 na
  z.nblk = (z.npos + crt_block_positions() - 1) / crt_block_positions();
  size_t off = 0;
  for (int i = 0; i < 3; ++i) {
    z.o_r[i] = off;
    off += align256(n2 * z.lc * 4);
  }
  z.o_pm = off;
  off += polymatmul_workspace_bytes(kIntPrimes[0], n, na);
  z.o_t = off;
  off += align256(n2 * z.nblk * crt_block_positions() * 8);
  z.o_blk = off;
  off += align256(n2 * z.nblk * 4);
  z.total = off;
  return z;
}

}  // namespace

extern "C" {

size_t intmatmul32_workspace_bytes(size_t n, size_t na) {
  if (!intmat_fits(n, na)) return 0;
  return intmat_layout(n, na).total;
}

int intmatmul_crt32(size_t n, const uint32_t* A, const uint32_t* B, size_t na, uint32_t* C, void* workspace,
                    size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    if (n == 0 || na == 0) return ok();
    if (!A || !B || !C) return fail(NTT_EINVAL, "NULL matrix pointer");
    if (!aligned_to(A, 4) || !aligned_to(B, 4) || !aligned_to(C, 4)) return fail(NTT_EINVAL, "misaligned pointer");
    if (n > kMatMaxN) return fail(NTT_EUNSUPPORTED, "n = %zu exceeds %u", n, kMatMaxN);
    if (!intmat_fits(n, na))
      return fail(NTT_EINVAL, "n = %zu, %zu chunks: coefficients could reach p1 p2 p3 or the transform exceed 2^23",
                  n, na);
    const IntMatLayout z = intmat_layout(n, na);
    if (ws_bytes < z.total || !workspace)
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", z.total, ws_bytes);
    unsigned char* w = (unsigned char*)workspace;
    const size_t n2 = n * n;
    for (int i = 0; i < 3; ++i) {
      // the polynomial matrix product modulo this prime; chunks of 32 bits exceed the
      // primes and are reduced as the first pass loads them
      int rc = polymat_run(kIntPrimes[i], n, A, B, na, w + z.o_r[i], w + z.o_pm, stream, true);
      if (rc) return rc;
    }
    CrtArgs x;
    memset(&x, 0, sizeof(x));
    crt_constants(&x);
    x.r1 = (const uint32_t*)(w + z.o_r[0]);
    x.r2 = (const uint32_t*)(w + z.o_r[1]);
    x.r3 = (const uint32_t*)(w + z.o_r[2]);
    x.lc = z.lc;
    x.npos = z.npos;
    x.t = (uint32_t*)(w + z.o_t);
    x.blk = (uint32_t*)(w + z.o_blk);
    x.c = C;
    x.rstride = z.lc;
    x.tstride = z.nblk * crt_block_positions();
    x.bstride = (uint32_t)z.nblk;
    x.cstride = z.npos;
    x.batch = (uint32_t)n2;
    HIP_TRY(launch_crt32_carry(x, stream));
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in intmatmul_crt32");
  }
}

}  // extern "C"

// ============================================================================ FP64 residues
namespace {

// Primes whose products over doubles take the kernels' band variant (2^49 <= p < 2^50:
// multiplicands reduced before each product).
bool f64_band(uint64_t p) { return p >= (1ull << 49); }

// Shape checks of one FP64 product: p < 2^50 prime; transforms up to 2^15 in one
// workgroup (fused), longer ones two-pass (columns of at most 2^10 words).
int f64_shape(const ntt_polymul_desc& d, size_t i, ProductShape* s) {
  if (d.p >= (1ull << 50))
    return fail(NTT_EUNSUPPORTED, "descriptor %zu: FP64 residues need p < 2^50", i);
  int rc = shape_of(d.p, d.la, d.lb, s);
  if (rc) {
    std::string m = g_last_error;
    return fail(rc, "descriptor %zu: %s", i, m.c_str());
  }
  s->wb = 64;
  s->fused = s->L <= fused_max_log2n(64);
  if (!s->fused && s->L - pass_max_row_log2(64) > 10)
    return fail(NTT_EUNSUPPORTED, "descriptor %zu: FP64 transform length 2^%d exceeds 2^%d", i, s->L,
                pass_max_row_log2(64) + 10);
  return NTT_OK;
}

}  // namespace

extern "C" {

int polymul_f64_batch_create(ntt_batch** out, const ntt_polymul_desc* d, size_t count) {
  try {
    if (!out) return fail(NTT_EINVAL, "out is NULL");
    *out = nullptr;
    if (g_capturing) return fail(NTT_EINVAL, "polymul_f64_batch_create allocates and cannot run during a graph capture");
    if (count && !d) return fail(NTT_EINVAL, "descriptor array is NULL");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<ProductShape> shapes(count);
    for (size_t i = 0; i < count; ++i) {
      if (d[i].la == 0 || d[i].lb == 0) {
        shapes[i].L = -1;
        continue;
      }
      if (!d[i].a || !d[i].b || !d[i].c) return fail(NTT_EINVAL, "descriptor %zu: NULL operand pointer", i);
      int rc = f64_shape(d[i], i, &shapes[i]);
      if (rc) return rc;
      if (!aligned_to(d[i].a, 8) || !aligned_to(d[i].b, 8) || !aligned_to(d[i].c, 8))
        return fail(NTT_EINVAL, "descriptor %zu: operands must be 8-byte aligned", i);
    }
    ntt_batch* bt = new ntt_batch();
    bt->device = dev;
    bt->ditems = nullptr;
    std::vector<FusedItem> items;
    for (int band = 0; band < 2; ++band) {
      for (int cls = 0; cls < kFusedClasses; ++cls) {
        const size_t first = items.size();
        for (size_t i = 0; i < count; ++i) {
          const ProductShape& s = shapes[i];
          if (s.L < 0 || !s.fused || fclass(64, s.L) != cls || f64_band(s.p) != (band != 0)) continue;
          ntt_plan* pl = nullptr;
          int rc = cached_plan(s.p, (uint32_t)s.L, &pl, true);
          if (rc) {
            delete bt;
            return rc;
          }
          items.push_back(fused_item(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c));
        }
        if (items.size() > first) bt->groups.push_back({band ? kF64BandGroup : kF64Group, cls, first, items.size() - first});
      }
    }
    for (size_t i = 0; i < count; ++i) {
      const ProductShape& s = shapes[i];
      if (s.L < 0 || s.fused) continue;
      ntt_plan* pl = nullptr;
      int rc = cached_plan(s.p, (uint32_t)s.L, &pl, true);
      if (rc) {
        delete bt;
        return rc;
      }
      bt->big.push_back({pl, d[i].a, d[i].b, d[i].c, d[i].la, d[i].lb, s.lc});
    }
    bt->cus = current_cus();
    bt->big_ws = batch_scratch(shapes, bt->cus, nullptr);
    if (!items.empty()) {
      if (hipMalloc(&bt->ditems, items.size() * sizeof(FusedItem)) != hipSuccess) {
        delete bt;
        return fail(NTT_ENOMEM, "hipMalloc of batch descriptors failed");
      }
      if (hipMemcpy(bt->ditems, items.data(), items.size() * sizeof(FusedItem), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(bt->ditems);
        delete bt;
        return fail(NTT_EDEVICE, "upload of batch descriptors failed");
      }
    }
    *out = bt;
    return ok();
  } catch (...) {
    return fail(NTT_ENOMEM, "exception in polymul_f64_batch_create");
  }
}

size_t polymul_f64_batch_workspace_bytes(const ntt_polymul_desc* d, size_t count) {
  if (!d && count) return 0;
  std::vector<ProductShape> shapes(count);
  for (size_t i = 0; i < count; ++i) {
    shapes[i].L = -1;
    if (d[i].la == 0 || d[i].lb == 0) continue;
    if (f64_shape(d[i], i, &shapes[i])) shapes[i].L = -1;
  }
  size_t nfused = 0;
  const size_t scratch = batch_scratch(shapes, current_cus(), &nfused);
  return align256(nfused * sizeof(FusedItem)) + scratch;
}

int polymul_f64_batch(const ntt_polymul_desc* d, size_t count, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    hipStream_t stream = (hipStream_t)hip_stream;
    if (capturing(stream))
      return fail(NTT_EINVAL, "polymul_f64_batch copies host descriptors and cannot be captured in a graph");
    if (count == 0) return ok();
    if (!d) return fail(NTT_EINVAL, "descriptor array is NULL");
    std::vector<ProductShape> shapes(count);
    for (size_t i = 0; i < count; ++i) {
      if (d[i].la == 0 || d[i].lb == 0) {
        shapes[i].L = -1;
        continue;
      }
      if (!d[i].a || !d[i].b || !d[i].c) return fail(NTT_EINVAL, "descriptor %zu: NULL operand pointer", i);
      int rc = f64_shape(d[i], i, &shapes[i]);
      if (rc) return rc;
      if (!aligned_to(d[i].a, 8) || !aligned_to(d[i].b, 8) || !aligned_to(d[i].c, 8))
        return fail(NTT_EINVAL, "descriptor %zu: operands must be 8-byte aligned", i);
    }
    const int cus = current_cus();
    size_t nfused = 0;
    const size_t scratch = batch_scratch(shapes, cus, &nfused);
    const size_t need = align256(nfused * sizeof(FusedItem)) + scratch;
    if (ws_bytes < need || (need && !workspace))
      return fail(NTT_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceCtx* ctx = device_ctx(dev);
    std::vector<FusedItem> items;
    items.reserve(nfused);
    struct Group { int cls; bool band; size_t first, count; };
    std::vector<Group> groups;
    for (int band = 0; band < 2; ++band) {
      for (int cls = 0; cls < kFusedClasses; ++cls) {
        const size_t first = items.size();
        for (size_t i = 0; i < count; ++i) {
          const ProductShape& s = shapes[i];
          if (s.L < 0 || !s.fused || fclass(64, s.L) != cls || f64_band(s.p) != (band != 0)) continue;
          ntt_plan* pl = nullptr;
          int rc = cached_plan(s.p, (uint32_t)s.L, &pl, true);
          if (rc) return rc;
          items.push_back(fused_item(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c));
        }
        if (items.size() > first) groups.push_back({cls, band != 0, first, items.size() - first});
      }
    }
    FusedItem* ditems = (FusedItem*)workspace;
    if (!items.empty()) {
      int rc = upload(ctx, ditems, items.data(), items.size() * sizeof(FusedItem), stream);
      if (rc) return rc;
    }
    void* bigws = (unsigned char*)workspace + align256(nfused * sizeof(FusedItem));
    for (const Group& g : groups) {
      FusedBatch fb;
      memset(&fb, 0, sizeof(fb));
      fb.items = ditems + g.first;
      fb.park = bigws;
      fb.count = (int)g.count;
      HIP_TRY(launch_fused_f64(g.cls, g.band, fb, fused_grid(64, g.cls, g.count, cus), stream));
    }
    // two-pass products (transforms above 2^15), one after the other in the scratch
    for (size_t i = 0; i < count; ++i) {
      const ProductShape& s = shapes[i];
      if (s.L < 0 || s.fused) continue;
      ntt_plan* pl = nullptr;
      int rc = cached_plan(s.p, (uint32_t)s.L, &pl, true);
      if (rc) return rc;
      rc = run_multipass_product(pl, d[i].a, d[i].la, d[i].b, d[i].lb, d[i].c, s.lc, false, bigws, stream);
      if (rc) return rc;
    }
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in polymul_f64_batch");
  }
}

}  // extern "C"

// ============================================================================ primitives alone
extern "C" {

int ntt_arith_apply(int op, int word, uint64_t p, const void* x, const void* y, const void* ys, uint64_t tw,
                    uint64_t tws, void* out, size_t n, void* hip_stream) {
  try {
    if (op < NTT_ARITH_SHOUP || op > NTT_ARITH_GS) return fail(NTT_EINVAL, "unknown primitive %d", op);
    if (word != 32 && word != 64 && word != 0) return fail(NTT_EINVAL, "word must be 32, 64 or 0 (doubles)");
    if (p < 3 || !(p & 1)) return fail(NTT_EINVAL, "modulus must be odd and at least 3");
    const uint64_t bound = word == 32 ? (1ull << 31) : word == 64 ? kMaxModulus : (1ull << 50);
    if (p >= bound) return fail(NTT_EUNSUPPORTED, "modulus %llu beyond the word's bound", (unsigned long long)p);
    if (n == 0) return ok();
    const bool needs_y = op != NTT_ARITH_RED1 && op != NTT_ARITH_RED2;
    if (!x || !out || (needs_y && !y) || (op == NTT_ARITH_SHOUP && word != 0 && !ys))
      return fail(NTT_EINVAL, "NULL array");
    const size_t esz = word == 32 ? 4 : 8;
    if (!aligned_to(x, esz) || !aligned_to(out, esz) || (y && !aligned_to(y, esz)) || (ys && !aligned_to(ys, esz)))
      return fail(NTT_EINVAL, "arrays must be %zu-byte aligned", esz);
    ArithArgs a;
    memset(&a, 0, sizeof(a));
    a.x = x;
    a.y = y;
    a.ys = ys;
    a.out = out;
    a.n = n;
    a.p = p;
    a.pinv = word ? inv_pow2_word(p, word) : 0;
    a.tw = tw;
    a.tws = tws;
    a.twd = (double)tw;
    a.op = op;
    a.word = word;
    HIP_TRY(launch_arith_apply(a, (hipStream_t)hip_stream));
    return ok();
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in ntt_arith_apply");
  }
}

}  // extern "C"

// ============================================================================ products without allocation
// polymul_modp for callers that cannot allocate device memory: its scratch (the park
// slice of the fused kernel, the partials of the split path, the two transformed
// operands of the two-pass path) lives in one fixed device array of this file.  Every
// device the library runs on holds its own copy of the array, at its own address, for
// the life of the process.  In host code the array's name is not a device address:
// the address is looked up once per device with hipGetSymbolAddress and only that
// address is handed to the kernels.
namespace {
constexpr size_t kStaticScratchBytes = NTT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NTT_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(NTT_EUNSUPPORTED, "device %d beyond the %d devices supported", dev,
                                                         kMaxScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(NTT_EDEVICE, "hipGetSymbolAddress of the static scratch on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NTT_OK;
}
}  // namespace

extern "C" {

int polymul_modp_noalloc(uint64_t p, const void* a, size_t la, const void* b, size_t lb, void* c, void* hip_stream) {
  try {
    if (la == 0 || lb == 0) return ok();
    ProductShape s;
    int rc = shape_of(p, la, lb, &s);
    if (rc) return rc;
    single_path(&s);
    const size_t need = single_product_ws(s, current_cus());
    if (need > kStaticScratchBytes)
      return fail(NTT_ENOMEM, "a product of transform length 2^%d needs %zu bytes of scratch, more than the %zu of "
                  "polymul_modp_noalloc", s.L, need, kStaticScratchBytes);
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return polymul_modp_run(p, a, la, b, lb, c, ws, kStaticScratchBytes, (hipStream_t)hip_stream, false,
                            "polymul_modp_noalloc");
  } catch (...) {
    return fail(NTT_EDEVICE, "exception in polymul_modp_noalloc");
  }
}

}  // extern "C"
