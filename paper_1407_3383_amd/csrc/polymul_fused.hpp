// Fused polynomial product kernels (section 5.2): fold, two forward transforms,
// entry-wise product, inverse transform and recombination, all inside one
// workgroup, for transform lengths up to 2^16 (32-bit) / 2^15 (64-bit) residues.
//
// A product of transform length N = 2^(d+M) runs as 2^d sub-problems of length
// 2^M = S that fit in LDS (two operands of S words each).  Sub-problem h starts
// from the fold f_h[j] = sum_k x[j + k S] psi_h^k (the first d forward stages,
// restricted to block h; psi_h = w_{2^d}^([h]_d)), is transformed, multiplied and
// inverse-transformed in LDS, and its result is parked (in registers, or in a
// per-workgroup slice of the workspace).  The last d inverse stages then combine
// the 2^d partial results position by position (each thread handles the same
// positions j of every partial) and the linear product is written out.  A launch
// loops over a descriptor list, so products of any prime and any length in the size
// class share one launch (section 2.2, Remark 6: several moduli in one vector launch).
#pragma once
#include <algorithm>

#include "kernels.hpp"
#include "ntt_wave.hpp"

namespace nttgpu {

// PM = 0: partials in registers; PM = 1: partials in the workspace slice `park`.
template <typename T, int LAZY, int NT, int M, int MAXD, int PM>
__device__ void polymul_item(const FusedItem& it, T* sa, T* sb, T* park_generic) {
  const gptr<T> park = gmut<T>(park_generic);
  const PolyConst<T>* __restrict__ pc = (const PolyConst<T>*)it.cst;
  Arith<T> ar;
  ar.p = pc->p;
  ar.p2 = pc->p2;
  ar.pinv = pc->pinv;
  const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(it.tw);
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(it.twi);
  const gcptr<T> a = gconst<T>(it.a);
  const gcptr<T> b = gconst<T>(it.b);
  const gptr<T> c = gmut<T>(it.c);
  constexpr int S = 1 << M;
  constexpr int EPT = (S + NT - 1) / NT;  // positions per thread
  const int d = (int)it.log2n - M;
  const int nsub = 1 << d;
  const uint64_t la = it.la, lb = it.lb, lc = la + lb - 1;
  // TFT truncation (d = 2): lc > 2S, so lam = ceil(lc / S) is 3 or 4; with 3 the fourth
  // partial is completed from the zero coefficients c_k, k >= 3S (plan constants tft2)
  const int lam = (d == 2 && lc <= 3 * (uint64_t)S) ? 3 : nsub;
  T P0[(PM == 0 && MAXD > 0) ? EPT : 1], P1[(PM == 0 && MAXD > 1) ? EPT : 1], P2[(PM == 0 && MAXD > 1) ? EPT : 1];
  T* const sv2[2] = {sa, sb};

  for (int h = 0; h < lam; ++h) {
    // Fold of both operands (indices >= la, lb read as 0); the Montgomery scale
    // 2^bits/N is applied to b so that the entry-wise Montgomery product yields
    // a^ b^ / N.  The terms k = 0, 1 of every position of the thread are requested
    // together (one HBM round trip); terms k >= 2 exist only when an operand is
    // longer than 2S and take a second loop.
    {
      const TwPair<T> fa1 = pc->fa[h][1], fb0 = pc->fb[h][0], fb1 = pc->fb[h][1];
      constexpr int FB = EPT < 8 ? EPT : 8;  // positions whose loads are in flight together
#pragma unroll 1
      for (int kb = 0; kb < EPT; kb += FB) {
        const int tf = opaque_tid() + kb * NT;
        T xa0[FB], xa1[FB], xb0[FB], xb1[FB];
#pragma unroll
        for (int k0 = 0; k0 < FB; ++k0) {
          const uint64_t j = (uint64_t)(tf + k0 * NT);
          const bool in = j < (uint64_t)S;
          xa0[k0] = (in && j < la) ? a[j] : (T)0;
          xb0[k0] = (in && j < lb) ? b[j] : (T)0;
          xa1[k0] = (in && nsub > 1 && j + S < la) ? a[j + S] : (T)0;
          xb1[k0] = (in && nsub > 1 && j + S < lb) ? b[j + S] : (T)0;
        }
#pragma unroll
        for (int k0 = 0; k0 < FB; ++k0) {
          const int j = tf + k0 * NT;
          if (j < S) {
            T fa = xa0[k0];
            T fb = ar.red1(ar.shoup(xb0[k0], fb0.w, fb0.ws));
            if (nsub > 1) {
              fa = ar.red1(fa + ar.red1(ar.shoup(xa1[k0], fa1.w, fa1.ws)));
              fb = ar.red1(fb + ar.red1(ar.shoup(xb1[k0], fb1.w, fb1.ws)));
            }
            if (nsub > 2 && (uint64_t)2 * S < (la > lb ? la : lb)) {
              for (int k = 2; k < nsub; ++k) {
                const uint64_t idx = (uint64_t)j + (uint64_t)k * S;
                if (idx < la) fa = ar.red1(fa + ar.red1(ar.shoup(a[idx], pc->fa[h][k].w, pc->fa[h][k].ws)));
                if (idx < lb) fb = ar.red1(fb + ar.red1(ar.shoup(b[idx], pc->fb[h][k].w, pc->fb[h][k].ws)));
              }
            }
            sa[lidx(j)] = fa;
            sb[lidx(j)] = fb;
          }
        }
      }
    }
    __syncthreads();
    if constexpr (M >= 10) {
      // Top M-10 stages across the workgroup, the other 10 inside each wave's
      // 1024-word block; the entry-wise product happens in registers between the
      // forward and the inverse wave-local rounds.
      fwd_G<T, LAZY, NT, 2, M>(ar, sv2, d, (uint32_t)h, tw);
      if ((opaque_tid() >> 6) < (1 << (M - 10))) {
        T x[2][16];
        fwd_W<T, LAZY, 2, M>(ar, sv2, d, (uint32_t)h, tw, x);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          T xa = x[0][i], yb = x[1][i];
          if constexpr (LAZY == kLazy) {
            xa = ar.red1(ar.red2(xa));  // xa < p, yb < 4p: xa yb < 2^bits p
          } else {  // xa < p, yb < 2p: xa yb < 2p^2 < 2^bits p (Function 13's bound)
            xa = ar.red1(xa);
            if constexpr (LAZY == kBand) yb = ar.red1(yb);  // Function 16 needs xa yb < 2^50 p
          }
          T z = ar.mont(xa, yb);  // (0, 2p)
          if constexpr (LAZY != kLazy) z = ar.red1(z);
          x[0][i] = z;
        }
        inv_W<T, LAZY, M>(ar, sa, d, (uint32_t)h, twi, x[0]);
      }
      inv_G<T, LAZY, NT, M>(ar, sa, d, (uint32_t)h, twi);
    } else {
      fwd_lds_ct<T, LAZY, NT, 2, M>(ar, sv2, d, (uint32_t)h, tw);
      const int tp = opaque_tid();
#pragma unroll 4
      for (int k0 = 0; k0 < EPT; ++k0) {
        const int j = tp + k0 * NT;
        if (j < S) {
          T x = sa[lidx(j)], y = sb[lidx(j)];
          if constexpr (LAZY == kLazy) {
            x = ar.red1(ar.red2(x));  // x < p, y < 4p: x y < 2^bits p
          } else {  // x < p, y < 2p: x y < 2p^2 < 2^bits p (Function 13's bound)
            x = ar.red1(x);
            if constexpr (LAZY == kBand) y = ar.red1(y);  // Function 16 needs x y < 2^50 p
          }
          T z = ar.mont(x, y);  // (0, 2p)
          if constexpr (LAZY != kLazy) z = ar.red1(z);
          sa[lidx(j)] = z;
        }
      }
      __syncthreads();
      inv_lds_ct<T, LAZY, NT, M>(ar, sa, d, (uint32_t)h, twi);
    }
    const int tr = opaque_tid();
    if (h + 1 < lam) {
      if constexpr (MAXD > 0) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {  // fully unrolled: P0..P2 stay in registers
          const int j = tr + k * NT;
          const T v = sa[lidx(j)];
          if constexpr (PM == 1) {
            park[(size_t)h * S + j] = v;
          } else {
            if (h == 0) P0[k] = v;
            else if (h == 1) P1[k] = v;
            else P2[k] = v;
          }
        }
      }
    } else {
      // Recombination: inverse global stages d-1 .. 0 across the partial results.
      T q0[EPT], q1[EPT], q2[EPT];
      if constexpr (PM == 1 && MAXD > 0) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {  // parked partials, one round trip
          const int j = tr + k * NT;
          q0[k] = (d >= 1) ? park[j] : (T)0;
          q1[k] = (d >= 2) ? park[S + j] : (T)0;
          q2[k] = (d >= 2) ? park[2 * S + j] : (T)0;
        }
      } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          q0[k] = (MAXD > 0) ? P0[k] : (T)0;
          q1[k] = (MAXD > 1) ? P1[k] : (T)0;
          q2[k] = (MAXD > 1) ? P2[k] : (T)0;
        }
      }
      // recombination twiddles and completion factors, loaded before any output store
      const TwPair<T> w1 = uni(ldtw<T>(twi + 1)), w2 = uni(ldtw<T>(twi + 2)), w3 = uni(ldtw<T>(twi + 3));
      TwPair<T> kf[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) kf[i] = uni(ldtw<T>(gconst<TwPair<T>>((const void*)&pc->tft2[i])));
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int j = tr + k * NT;
        if (j < S) {
          T v0 = sa[lidx(j)];
          const uint64_t jj = (uint64_t)j;
          if (d == 0) {
            if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, v0);
          } else if (d == 1) {
            if constexpr (MAXD > 0) {
              T x = q0[k];
              gs_bfly<LAZY, true>(ar, x, v0, w1);
              if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, x);
              if (jj + S < lc) c[jj + S] = canon_from_inv<LAZY>(ar, v0);
            }
          } else {
            if constexpr (MAXD > 1) {
              T x0 = q0[k], x1 = q1[k], x2, x3;
              if (lam == 4) {
                x2 = q2[k];
                x3 = v0;
              } else {  // x3 = k0 x0 + k1 x1 + k2 x2: the partial that makes c_3 vanish
                x2 = v0;
                const T s0 = ar.red1(ar.shoup_u(x0, kf[0].w, kf[0].ws));
                const T s1 = ar.red1(ar.shoup_u(x1, kf[1].w, kf[1].ws));
                const T s2 = ar.red1(ar.shoup_u(x2, kf[2].w, kf[2].ws));
                x3 = ar.red1(ar.red1(s0 + s1) + s2);
              }
              gs_bfly<LAZY, true>(ar, x0, x1, w2);
              gs_bfly<LAZY, true>(ar, x2, x3, w3);
              gs_bfly<LAZY, true>(ar, x0, x2, w1);
              gs_bfly<LAZY, true>(ar, x1, x3, w1);
              if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, x0);
              if (jj + S < lc) c[jj + S] = canon_from_inv<LAZY>(ar, x1);
              if (jj + 2 * (uint64_t)S < lc) c[jj + 2 * (uint64_t)S] = canon_from_inv<LAZY>(ar, x2);
              if (jj + 3 * (uint64_t)S < lc) c[jj + 3 * (uint64_t)S] = canon_from_inv<LAZY>(ar, x3);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// Wave-local variant (10 <= M <= 14, NT = 2^(M-4) threads doing wave work).
// Per sub-problem: one "boundary" phase and one wave phase, two barriers.
//  boundary(h): for each of the thread's clusters {q + 1024 c}:
//     - request the fold inputs of sub-problem h (the same positions for every h),
//     - finish sub-problem h-1: its top inverse stages (G'), then park the partial or,
//       after the last one, recombine with the parked partials and store c,
//     - fold sub-problem h, run its top forward stages (G) on both operands, store
//       the clusters to LDS;
//  wave(h): the wave-local forward rounds of both operands, the entry-wise
//     product in registers and the wave-local inverse rounds.
// G'(h-1) and G(h) touch the same elements of the same thread, so no barrier
// separates them, and the fold loads are in flight while G' computes.
template <typename T, int LAZY, int NT, int M, int MAXD>
__device__ __forceinline__ void polymul_item_wave(const FusedItem& it_in, T* sa, T* sb, T* park_generic) {
  static_assert(M >= 10 && M <= 14, "wave-local sub-problems span 2^10 .. 2^14 words");
  // the descriptor is the same for the whole workgroup: keep it in scalar registers
  FusedItem it;
  it.a = uni(it_in.a);
  it.b = uni(it_in.b);
  it.c = uni(it_in.c);
  it.la = uni((uint64_t)it_in.la);
  it.lb = uni((uint64_t)it_in.lb);
  it.cst = uni(it_in.cst);
  it.tw = uni(it_in.tw);
  it.twi = uni(it_in.twi);
  it.log2n = uni(it_in.log2n);
  const gptr<T> park = gmut<T>(uni((void*)park_generic));
  const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(it.cst);
  Arith<T> ar;
  ar.p = uni(pc->p);
  ar.p2 = uni(pc->p2);
  ar.pinv = uni(pc->pinv);
  const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(it.tw);
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(it.twi);
  const gcptr<T> a = gconst<T>(it.a);
  const gcptr<T> b = gconst<T>(it.b);
  const gptr<T> c = gmut<T>(it.c);
  constexpr int S = 1 << M;
  constexpr int R = M - 10;           // top stages done across the workgroup
  constexpr int C = 1 << R;           // elements per top-stage cluster
  constexpr int CPT = 1024 / NT > 0 ? 1024 / NT : 1;  // clusters per thread
  constexpr int EPT = CPT * C;        // positions per thread
  const int d = (int)it.log2n - M;
  const int nsub = 1 << d;
  const uint64_t la = it.la, lb = it.lb, lc = la + lb - 1;
  const bool more_terms = nsub > 2 && (uint64_t)2 * S < (la > lb ? la : lb);
  // TFT truncation: only the sub-problems h < lam hold outputs below lc; the last
  // partial is completed from the zero coefficients when lam < nsub (d = 2, lam = 3)
  const int lam = (int)((lc + S - 1) / S < (uint64_t)nsub ? (lc + S - 1) / S : (uint64_t)nsub);
  T* const sv2[2] = {sa, sb};
  // the wave-local rounds request their twiddles a round ahead (fwd_W / inv_W with PF)
  constexpr bool kWavePF = true;

  // G' (top inverse stages) of sub-problem hp on the thread's clusters, with its
  // twiddles wi (requested by finish_twiddles ahead of the operand loads, through
  // scalar loads whose wait does not include those loads); hands each finished value
  // to `sink(e, j, value)`.
  auto finish_twiddles = [&](TwPair<T>* wi, int hp) {
    if constexpr (R > 0) cluster_twiddles<T, R, true, true>(wi, twi, d, 0, (uint32_t)hp, 0u);
  };
  auto finish = [&](const TwPair<T>* wi, int t0, auto&& sink) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = t0 + i * NT;
      const int lb0 = lidx(q);
      T v[C];
#pragma unroll
      for (int cc = 0; cc < C; ++cc) v[cc] = sa[lb0 + cc * 1056];
      if constexpr (R > 0) cluster_inv<T, LAZY, R, true>(ar, v, wi);
#pragma unroll
      for (int cc = 0; cc < C; ++cc) sink(i * C + cc, q + 1024 * cc, v[cc]);
    }
  };

  // Fold inputs: the same positions of a and b for every sub-problem.  They are
  // requested at the start of the boundary phase of h and are in flight while G' of
  // h - 1 computes and parks.  Requested earlier (during the wave phase) they would
  // be live across it and spill.  When both operands cover [0, 2S) the loads carry no
  // predicates: they issue as one burst, without a branch per load.
  T x0[EPT], x1[EPT], y0[EPT], y1[EPT];
  const bool full2 = nsub > 1 && la >= (uint64_t)2 * S && lb >= (uint64_t)2 * S;
  auto request_fold_inputs = [&]() {
    const int tq = opaque_tid();
    if (full2) {
#pragma unroll
      for (int i = 0; i < CPT; ++i)
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          const int e = i * C + cc;
          const uint32_t j = (uint32_t)(tq + i * NT) + 1024u * cc;
          x0[e] = a[j];
          y0[e] = b[j];
          x1[e] = a[j + S];
          y1[e] = b[j + S];
        }
      return;
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i)
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        const int e = i * C + cc;
        const uint64_t j = (uint64_t)(tq + i * NT) + 1024u * cc;
        x0[e] = j < la ? a[j] : (T)0;
        y0[e] = j < lb ? b[j] : (T)0;
        x1[e] = (nsub > 1 && j + S < la) ? a[j + S] : (T)0;
        y1[e] = (nsub > 1 && j + S < lb) ? b[j + S] : (T)0;
      }
  };
  for (int h = 0; h < lam; ++h) {
    const int t0 = opaque_tid();
    // ---- boundary phase: G' of h-1 and park, fold + G of h.  G''s twiddles (scalar
    // loads, requested for every h so that no branch separates them from their use)
    // go out before the operands, the fold's after G' (their scalar registers are not
    // live at the same time).
    TwPair<T> wi[C > 1 ? C - 1 : 1];
    if constexpr (MAXD > 0) finish_twiddles(wi, h > 0 ? h - 1 : 0);
    request_fold_inputs();
    if constexpr (MAXD > 0) {
      if (h > 0) finish(wi, t0, [&](int, int j, T v) { park[(size_t)(h - 1) * S + j] = v; });
    }
    {
      const gcptr<TwPair<T>> fah = &pc->fa[h][0], fbh = &pc->fb[h][0];
      const TwPair<T> fa1 = ldtw_s<T>(fah + 1), fb0 = ldtw_s<T>(fbh), fb1 = ldtw_s<T>(fbh + 1);
      TwPair<T> wf[C > 1 ? C - 1 : 1];
      if constexpr (R > 0) cluster_twiddles<T, R, true, true>(wf, tw, d, 0, (uint32_t)h, 0u);
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int q = t0 + i * NT;
        T v[2][C];
        if (nsub > 1 && !more_terms) {  // two terms per position: no branch per position
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            const int e = i * C + cc;
            v[0][cc] = ar.red1(x0[e] + ar.red1(ar.shoup_u(x1[e], fa1.w, fa1.ws)));
            v[1][cc] = ar.red1(ar.red1(ar.shoup_u(y0[e], fb0.w, fb0.ws)) + ar.red1(ar.shoup_u(y1[e], fb1.w, fb1.ws)));
          }
        } else {
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            const int e = i * C + cc;
            T fa = x0[e];
            T fb = ar.red1(ar.shoup_u(y0[e], fb0.w, fb0.ws));
            if (nsub > 1) {
              fa = ar.red1(fa + ar.red1(ar.shoup_u(x1[e], fa1.w, fa1.ws)));
              fb = ar.red1(fb + ar.red1(ar.shoup_u(y1[e], fb1.w, fb1.ws)));
            }
            if (more_terms) {
              const uint64_t j = (uint64_t)q + 1024u * cc;
              for (int k = 2; k < nsub; ++k) {
                const uint64_t idx = j + (uint64_t)k * S;
                if (idx < la) {
                  const TwPair<T> f = ldtw<T>(&pc->fa[h][k]);
                  fa = ar.red1(fa + ar.red1(ar.shoup(a[idx], f.w, f.ws)));
                }
                if (idx < lb) {
                  const TwPair<T> f = ldtw<T>(&pc->fb[h][k]);
                  fb = ar.red1(fb + ar.red1(ar.shoup(b[idx], f.w, f.ws)));
                }
              }
            }
            v[0][cc] = fa;
            v[1][cc] = fb;
          }
        }
        if constexpr (R > 0) cluster_fwd<T, LAZY, R, 2, true>(ar, v, 0, wf);
        const int lb0 = lidx(q);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          sa[lb0 + cc * 1056] = v[0][cc];
          sb[lb0 + cc * 1056] = v[1][cc];
        }
      }
    }
    __syncthreads();
    // ---- wave phase
    if ((opaque_tid() >> 6) < (1 << (M - 10))) {
      T x[2][16];
      fwd_W<T, LAZY, 2, M, kWavePF>(ar, sv2, d, (uint32_t)h, tw, x);
      InvWTw<T> itw;
      if constexpr (kWavePF) inv_W_twiddles<T, M>(itw, d, (uint32_t)h, twi);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        T xa = x[0][i], yb = x[1][i];
        if constexpr (LAZY == kLazy) {
          xa = ar.red1(ar.red2(xa));  // xa < p, yb < 4p: xa yb < 2^bits p
        } else {  // xa < p, yb < 2p: xa yb < 2p^2 < 2^bits p (Function 13's bound)
          xa = ar.red1(xa);
          if constexpr (LAZY == kBand) yb = ar.red1(yb);  // Function 16 needs xa yb < 2^50 p
        }
        T z = ar.mont(xa, yb);  // (0, 2p)
        if constexpr (LAZY != kLazy) z = ar.red1(z);
        x[0][i] = z;
      }
      inv_W<T, LAZY, M, kWavePF>(ar, sa, d, (uint32_t)h, twi, x[0], -1, &itw);
    }
    __syncthreads();
  }
  // ---- last boundary: G' of the last sub-problem and the recombination
  {
    const int t0 = opaque_tid();
    // Recombination twiddles and completion factors first (from L2), then the parked
    // partials, all before any output store (a load placed after a store would wait
    // for the store as well).  Each partial's loads form one block under one uniform
    // test, not a branch per load (a branch per load makes every join wait for all
    // loads in flight).
    TwPair<T> wi[C > 1 ? C - 1 : 1];
    finish_twiddles(wi, lam - 1);
    TwPair<T> w1, w2, w3, k0, k1, k2;
    if constexpr (MAXD > 0) {
      const gcptr<TwPair<T>> kt = &pc->tft2[0];
      w1 = ldtw_s<T>(twi + 1);
      w2 = ldtw_s<T>(twi + 2);
      w3 = ldtw_s<T>(twi + 3);
      k0 = ldtw_s<T>(kt);
      k1 = ldtw_s<T>(kt + 1);
      k2 = ldtw_s<T>(kt + 2);
    }
    T q0[EPT], q1[EPT], q2[EPT];
    if constexpr (MAXD > 0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) q0[e] = q1[e] = q2[e] = (T)0;
      auto load_partial = [&](T(&q)[EPT], int k) {
#pragma unroll
        for (int i = 0; i < CPT; ++i)
#pragma unroll
          for (int cc = 0; cc < C; ++cc) q[i * C + cc] = park[(size_t)k * S + (t0 + i * NT + 1024 * cc)];
      };
      if (d >= 1) load_partial(q0, 0);
      if (d >= 2) load_partial(q1, 1);
      if (d >= 2 && lam == 4) load_partial(q2, 2);
    }
    finish(wi, t0, [&](int e, int j, T v) {
      const uint64_t jj = (uint64_t)j;
      if (d == 0) {
        if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, v);
      } else if (d == 1) {
        if constexpr (MAXD > 0) {
          T u0 = q0[e], u1 = v;
          gs_bfly<LAZY, true>(ar, u0, u1, w1);
          if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, u0);
          if (jj + S < lc) c[jj + S] = canon_from_inv<LAZY>(ar, u1);
        }
      } else {
        if constexpr (MAXD > 1) {
          T u0 = q0[e], u1 = q1[e], u2, u3;
          if (lam == 4) {
            u2 = q2[e];
            u3 = v;
          } else {  // u3 = k0 u0 + k1 u1 + k2 u2: the partial that makes c_3 vanish
            u2 = v;
            const T s0 = ar.red1(ar.shoup_u(u0, k0.w, k0.ws)), s1 = ar.red1(ar.shoup_u(u1, k1.w, k1.ws));
            const T s2 = ar.red1(ar.shoup_u(u2, k2.w, k2.ws));
            u3 = ar.red1(ar.red1(s0 + s1) + s2);
          }
          gs_bfly<LAZY, true>(ar, u0, u1, w2);
          gs_bfly<LAZY, true>(ar, u2, u3, w3);
          gs_bfly<LAZY, true>(ar, u0, u2, w1);
          gs_bfly<LAZY, true>(ar, u1, u3, w1);
          if (lc >= (uint64_t)4 * S - 1) {  // every output but possibly the very last one exists
            const uint32_t j32 = (uint32_t)j;
            c[j32] = canon_from_inv<LAZY>(ar, u0);
            c[j32 + S] = canon_from_inv<LAZY>(ar, u1);
            c[j32 + 2 * S] = canon_from_inv<LAZY>(ar, u2);
            if (j32 + 3 * S < (uint32_t)lc) c[j32 + 3 * S] = canon_from_inv<LAZY>(ar, u3);
          } else {
            if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, u0);
            if (jj + S < lc) c[jj + S] = canon_from_inv<LAZY>(ar, u1);
            if (jj + 2 * (uint64_t)S < lc) c[jj + 2 * (uint64_t)S] = canon_from_inv<LAZY>(ar, u2);
            if (jj + 3 * (uint64_t)S < lc) c[jj + 3 * (uint64_t)S] = canon_from_inv<LAZY>(ar, u3);
          }
        }
      }
    });
    __syncthreads();
  }
}

// Products of transform length 2^16 over 32-bit words as two sub-problems of 2^15
// points (d = 1) in one workgroup of 1024 threads.  LDS holds one operand's
// sub-problem (2^15 words), so the first operand's transform stays in registers (two
// 1024-word blocks per wave, 32 words per thread) while the second is transformed in
// LDS; the entry-wise product and the inverse then run as in polymul_item_wave.
// Against four sub-problems of 2^14 this reads each operand twice instead of four
// times, parks one partial instead of three, and its fold is one addition (the
// sub-problem inputs are a_lo + a_hi and a_lo - a_hi, or the operand itself when it
// has at most 2^15 coefficients).  Per sub-problem h:
//   A: fold of a, top 5 stages (radix-32 clusters at stride 1024), LDS;  barrier;
//      wave-local rounds of the wave's two blocks, kept in registers;    barrier;
//   B: the same for b (scaled by sigma);                                  barrier;
//      wave-local rounds of b, entry-wise product, wave-local inverse;    barrier;
//   G': top 5 inverse stages; park (h = 0) or recombine with the parked partial.
// HI: an operand may have more than 2^15 coefficients (a fold of two halves).
template <typename T, int LAZY, bool HI>
__device__ __forceinline__ void polymul_item_w15(const FusedItem& it_in, T* sa, T* park_generic) {
  constexpr int M = 15, S = 1 << M, C = 32, d = 1;
  FusedItem it;
  it.a = uni(it_in.a);
  it.b = uni(it_in.b);
  it.c = uni(it_in.c);
  it.la = uni((uint64_t)it_in.la);
  it.lb = uni((uint64_t)it_in.lb);
  it.cst = uni(it_in.cst);
  it.tw = uni(it_in.tw);
  it.twi = uni(it_in.twi);
  const gptr<T> park = gmut<T>(uni((void*)park_generic));
  const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(it.cst);
  Arith<T> ar;
  ar.p = uni(pc->p);
  ar.p2 = uni(pc->p2);
  ar.pinv = uni(pc->pinv);
  const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(it.tw);
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(it.twi);
  const gcptr<T> a = gconst<T>(it.a);
  const gcptr<T> b = gconst<T>(it.b);
  const gptr<T> c = gmut<T>(it.c);
  const uint64_t la = it.la, lb = it.lb, lc = la + lb - 1;
  const int wave = __builtin_amdgcn_readfirstlane(opaque_tid() >> 6);
  // Montgomery scale of the entry-wise product (2^32 / N), applied to b's inputs
  const TwPair<T> sig = ldtw_s<T>(&pc->fb[0][0]);

  // fold inputs of one operand, requested ahead: lo[c] = x[q + 1024 c] (the upper
  // half, x[q + 1024 c + S], is read where it is added: HI items are rare, and holding
  // both halves across a phase would spill)
  T lo[C];
  auto request = [&](gcptr<T> x, uint64_t len) {
    const int q = opaque_tid();
    if (len >= (uint64_t)S) {
#pragma unroll
      for (int cc = 0; cc < C; ++cc) lo[cc] = x[q + 1024 * cc];
    } else {
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        const uint32_t j = (uint32_t)(q + 1024 * cc);
        lo[cc] = j < len ? x[j] : (T)0;
      }
    }
  };
  // fold (u = lo + hi or lo - hi), optional scale, top 5 forward stages, store to LDS
  auto top_forward = [&](int h, gcptr<T> x, uint64_t len, bool scale) {
    const int q = opaque_tid();
    T v[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) {
      T u = lo[cc];
      if constexpr (HI) {
        const uint64_t j = (uint64_t)(q + 1024 * cc) + S;
        const T hv = j < len ? x[j] : (T)0;
        u = h == 0 ? ar.red1(u + hv) : ar.red1(u - hv + ar.p);
      }
      if (scale) u = ar.red1(ar.shoup_u(u, sig.w, sig.ws));
      v[cc] = u;
    }
    // cluster stage u pairs (cc, cc + 2^(4-u)) with TW[2^(d+u) + (h << u) + vv], vv = cc >> (5-u)
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int half = 16 >> u;
#pragma unroll
      for (int vv = 0; vv < (1 << u); ++vv) {
        const TwPair<T> ww = ldtw_s<T>(tw + ((1u << (d + u)) + ((uint32_t)h << u) + (uint32_t)vv));
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int cc = (vv << (5 - u)) + c2;
          ct_bfly<LAZY, true>(ar, v[cc], v[cc + half], ww);
        }
      }
    }
    const int lb0 = lidx(q);
#pragma unroll
    for (int cc = 0; cc < C; ++cc) sa[lb0 + cc * 1056] = v[cc];
  };

  request(a, la);
  // (the wave-local rounds here do not request their twiddles ahead: with the
  // operand a's transform held in registers that would spill 312 bytes per lane)
  for (int h = 0; h < 2; ++h) {
    // ---- A: fold, top stages, wave-local rounds kept in registers
    top_forward(h, a, la, false);
    __syncthreads();
    T xa[2][16];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      T* const sv1[1] = {sa};
      T x[1][16];
      fwd_W<T, LAZY, 1, M>(ar, sv1, d, (uint32_t)h, tw, x, wave + 16 * k);
#pragma unroll
      for (int i = 0; i < 16; ++i) xa[k][i] = x[0][i];
    }
    __syncthreads();
    // ---- B: fold, scale, top stages; wave-local rounds, entry-wise product, inverse
    request(b, lb);
    top_forward(h, b, lb, true);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      T* const sv1[1] = {sa};
      T x[1][16];
      fwd_W<T, LAZY, 1, M>(ar, sv1, d, (uint32_t)h, tw, x, wave + 16 * k);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        T xv = xa[k][i], yv = x[0][i];
        if constexpr (LAZY == kLazy) {
          xv = ar.red1(ar.red2(xv));  // xv < p, yv < 4p: xv yv < 2^bits p
        } else {  // xv < p, yv < 2p: xv yv < 2p^2 < 2^bits p (Function 13's bound)
          xv = ar.red1(xv);
          if constexpr (LAZY == kBand) yv = ar.red1(yv);  // Function 16 needs xv yv < 2^50 p
        }
        T z = ar.mont(xv, yv);  // (0, 2p)
        if constexpr (LAZY != kLazy) z = ar.red1(z);
        x[0][i] = z;
      }
      inv_W<T, LAZY, M>(ar, sa, d, (uint32_t)h, twi, x[0], wave + 16 * k);
    }
    __syncthreads();
    // ---- G': top 5 inverse stages; the next sub-problem's a is requested first
    if (h == 0) request(a, la);
    {
      const int q = opaque_tid();
      const int lb0 = lidx(q);
      T v[C];
#pragma unroll
      for (int cc = 0; cc < C; ++cc) v[cc] = sa[lb0 + cc * 1056];
#pragma unroll
      for (int u = 4; u >= 0; --u) {
        const int half = 16 >> u;
#pragma unroll
        for (int vv = 0; vv < (1 << u); ++vv) {
          const TwPair<T> ww = ldtw_s<T>(twi + ((1u << (d + u)) + ((uint32_t)h << u) + (uint32_t)vv));
#pragma unroll
          for (int c2 = 0; c2 < half; ++c2) {
            const int cc = (vv << (5 - u)) + c2;
            gs_bfly<LAZY, true>(ar, v[cc], v[cc + half], ww);
          }
        }
      }
      if (h == 0) {
#pragma unroll
        for (int cc = 0; cc < C; ++cc) park[q + 1024 * cc] = v[cc];
      } else {
        // the last inverse stage across the two partials: (u0, u1) -> (u0 + u1, (u0 - u1) w)
        const TwPair<T> w1 = ldtw_s<T>(twi + 1);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          const uint32_t j = (uint32_t)(q + 1024 * cc);
          T u0 = park[j], u1 = v[cc];
          gs_bfly<LAZY, true>(ar, u0, u1, w1);
          if (lc >= (uint64_t)2 * S - 1) {  // every output but possibly the last one exists
            c[j] = canon_from_inv<LAZY>(ar, u0);
            if (j + S < (uint32_t)lc) c[j + S] = canon_from_inv<LAZY>(ar, u1);
          } else {
            if (j < lc) c[j] = canon_from_inv<LAZY>(ar, u0);
            if ((uint64_t)j + S < lc) c[j + S] = canon_from_inv<LAZY>(ar, u1);
          }
        }
      }
    }
  }
  __syncthreads();
}

// The arithmetic mode of the item's prime: kLazy or kSafe read from its constants, or
// kBand in the kernels instantiated for residues in doubles with 2^49 <= p < 2^50 (a
// kernel of their own, so that the extra reductions do not weigh on the register
// allocation of the other two modes).
template <typename T, int NT, int M, int MAXD, int PM, bool BAND>
__device__ __forceinline__ void polymul_dispatch_lazy(const FusedItem& it, T* sa, T* sb, T* park) {
  const PolyConst<T>* pc = (const PolyConst<T>*)it.cst;
  if constexpr (M == 15) {  // 32-bit words, transform length 2^16 (d = 1), no band
    static_assert(NT == 1024 && !BAND && sizeof(T) == 4, "2^15-point sub-problems: 32-bit words, 1024 threads");
    const bool hi = uni((uint64_t)it.la) > (1u << 15) || uni((uint64_t)it.lb) > (1u << 15);
    if (uni(gconst<PolyConst<T>>(uni(it.cst))->lazy)) {
      if (hi) polymul_item_w15<T, kLazy, true>(it, sa, park);
      else polymul_item_w15<T, kLazy, false>(it, sa, park);
    } else {
      if (hi) polymul_item_w15<T, kSafe, true>(it, sa, park);
      else polymul_item_w15<T, kSafe, false>(it, sa, park);
    }
  } else if constexpr (BAND) {
    if constexpr (M >= 10 && PM == 1) polymul_item_wave<T, kBand, NT, M, MAXD>(it, sa, sb, park);
    else polymul_item<T, kBand, NT, M, MAXD, PM>(it, sa, sb, park);
  } else if constexpr (M >= 10 && PM == 1) {
    if (uni(gconst<PolyConst<T>>(uni(it.cst))->lazy)) polymul_item_wave<T, kLazy, NT, M, MAXD>(it, sa, sb, park);
    else polymul_item_wave<T, kSafe, NT, M, MAXD>(it, sa, sb, park);
  } else {
    if (pc->lazy) polymul_item<T, kLazy, NT, M, MAXD, PM>(it, sa, sb, park);
    else polymul_item<T, kSafe, NT, M, MAXD, PM>(it, sa, sb, park);
  }
}

// Sub-problem size 2^M for a product of transform length 2^L in a class whose
// largest sub-problem is 2^LOGS and smallest transform 2^LMIN.
template <typename T, int NT, int LOGS, int LMIN, int MAXD, int PM, bool BAND>
__device__ __forceinline__ void polymul_dispatch(const FusedItem& it, T* sa, T* sb, T* park) {
  const int L = (int)it.log2n;
  const int m = L < LOGS ? L : LOGS;
  if constexpr (LOGS - LMIN >= 10) {
    if (m <= LOGS - 10) { polymul_dispatch_lazy<T, NT, LOGS - 10, MAXD, PM, BAND>(it, sa, sb, park); return; }
  }
#define NTT_CASE(K)                                                                    \
  if constexpr (LOGS - LMIN >= K) {                                                    \
    if (m == LOGS - K) { polymul_dispatch_lazy<T, NT, LOGS - K, MAXD, PM, BAND>(it, sa, sb, park); return; } \
  }
  NTT_CASE(9) NTT_CASE(8) NTT_CASE(7) NTT_CASE(6) NTT_CASE(5) NTT_CASE(4) NTT_CASE(3) NTT_CASE(2) NTT_CASE(1)
#undef NTT_CASE
  polymul_dispatch_lazy<T, NT, LOGS, MAXD, PM, BAND>(it, sa, sb, park);
}

// Workgroup w serves items w, w + G, w + 2G, ...; with PM = 1 it parks partial
// results in its own workspace slice of 3 * 2^LOGS words.  BAND: every item is a
// product over doubles with 2^49 <= p < 2^50.
template <typename T, int NT, int LOGS, int LMIN, int MAXD, int PM, bool BAND = false>
__global__ __launch_bounds__(NT) void polymul_fused_kernel(FusedBatch batch) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sa = (T*)smem_raw;
  T* sb = LOGS == 15 ? nullptr : sa + lds_words(1 << LOGS);
  T* park = PM == 1 ? (T*)batch.park + (size_t)blockIdx.x * (LOGS == 15 ? 1 : 3) * ((size_t)1 << LOGS) : nullptr;
  for (int i = blockIdx.x; i < batch.count; i += gridDim.x) {
    const FusedItem it = batch.items ? batch.items[i] : batch.single;
    polymul_dispatch<T, NT, LOGS, LMIN, MAXD, PM, BAND>(it, sa, sb, park);
  }
}

template <typename T, int NT, int LOGS, int LMIN, int MAXD, int PM, bool BAND = false>
hipError_t launch_fused_cls(const FusedBatch& batch, int grid, hipStream_t stream) {
  // two operands' sub-problems in LDS, one for 2^15-point sub-problems
  const size_t lds = (LOGS == 15 ? 1 : 2) * (size_t)lds_words(1 << LOGS) * sizeof(T);
  auto k = polymul_fused_kernel<T, NT, LOGS, LMIN, MAXD, PM, BAND>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, batch);
  return hipGetLastError();
}

// One translation unit per word type and class group (compiled in parallel).
hipError_t launch_fused_w32_small(int cls, const FusedBatch& batch, int grid, hipStream_t stream);
hipError_t launch_fused_w32_c3(const FusedBatch& batch, int grid, hipStream_t stream);
hipError_t launch_fused_w32_c4(const FusedBatch& batch, int grid, hipStream_t stream);
hipError_t launch_fused_w64(int cls, const FusedBatch& batch, int grid, hipStream_t stream);

}  // namespace nttgpu
