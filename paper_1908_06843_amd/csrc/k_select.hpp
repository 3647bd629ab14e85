// Exact per-point selection shared by the projection kernels: radix select
// over order-preserving keys, and the band re-scoring with a compensated
// FP32 dot product that makes the selection exact with respect to the real
// scores (ties to the lower latent index, near-ties flagged).
#pragma once

#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

template <int RM>
__device__ __forceinline__ void radix_select(const uint32_t (&key)[RM], int R, int k,
                                             uint64_t (&selm)[RM]) {
  // T = the k-th largest key: the largest t with #{key >= t} >= k, built
  // bit by bit; stops early once a prefix isolates exactly k keys.
  uint32_t T = 0;
  bool exact = false;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t cand = T | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < RM; ++i)
      if (i < R) cnt += __popcll(ballot64(key[i] >= cand));
    if (cnt >= k) {
      T = cand;
      if (cnt == k) {
        exact = true;
        break;
      }
    }
  }
  if (exact) {
#pragma unroll
    for (int i = 0; i < RM; ++i) selm[i] = (i < R) ? ballot64(key[i] >= T) : 0ull;
    return;
  }
  int cgt = 0;
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    selm[i] = (i < R) ? ballot64(key[i] > T) : 0ull;
    cgt += __popcll(selm[i]);
  }
  int need = k - cgt;  // ties at T, lowest latent index first
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    if (i < R) {
      uint64_t eq = ballot64(key[i] == T);
      while (need > 0 && eq) {
        uint64_t low = eq & (~eq + 1ull);
        selm[i] |= low;
        eq &= eq - 1ull;
        --need;
      }
    }
  }
}

// Running list of the KL largest values (descending) without indices:
// a new value bubbles down by max/min pairs.
template <int KL>
__device__ __forceinline__ void list_insert(float (&t)[KL], float v) {
  static_for<0, KL>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const float hi = fmaxf(t[k], v);
    v = fminf(t[k], v);
    t[k] = hi;
  });
}

template <int KL>
__device__ __forceinline__ float list_at(const float (&t)[KL], int i) {
  float r = t[0];
  static_for<1, KL>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    r = (i == k) ? t[k] : r;
  });
  return r;
}

// Sum over the 64 lanes of RPW per-lane values at once (butterfly
// reduce-scatter): afterwards lanes whose index is a multiple of 64/RPW hold
// the total of value `row` (returned).
template <int RPW>
__device__ __forceinline__ int wave_sum_rows(double (&v)[RPW], int lane, double& total) {
  int row = 0;
  static_for<0, 6>([&](auto sc) {
    constexpr int st = decltype(sc)::value;
    constexpr int off = 32 >> st;
    constexpr int half = RPW >> (st + 1);
    if constexpr (half >= 1) {
      const bool upper = (lane & off) != 0;
      static_for<0, half>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double keep = upper ? v[i + half] : v[i];
        const double send = upper ? v[i] : v[i + half];
        v[i] = keep + __shfl_xor(send, off, 64);
      });
      if (upper) row += half;
    } else {
      v[0] += __shfl_xor(v[0], off, 64);
    }
  });
  total = v[0];
  return row;
}

// Score modes of the selection: the singleton log-joint of latent h up to
// latent-independent terms and the factor 1/sigma^2, from b_h and the half
// norm hn_h = 1/2 ||P_h||^2:
//   SCORE_LIN  b - hn                      (BSC, MCA, MMCA)
//   SCORE_ABS  |b| - hn                    (TSC: the better sign)
//   SCORE_DSC  max_{v >= 1} cs_v + phi_v b - phi_v^2 hn
//              (DSC: the best non-zero value, cs_v = sigma^2 ln(pv_v/pv_0))
enum { SCORE_LIN = 0, SCORE_ABS = 1, SCORE_DSC = 2 };

__device__ __forceinline__ float dsc_score(const Theta* __restrict__ th, float b, float hnh,
                                           float hnl) {
  const int nv = th->nv;
  const float hn = hnh + hnl;
  float r = -INFINITY;
#pragma unroll
  for (int v = 1; v < DSC_MAXV; ++v) {
    if (v < nv) {
      const float ph = th->phi[v];
      r = fmaxf(r, (th->cs[v] + ph * b) - (ph * ph) * hn);
    }
  }
  return r;
}

// The same from a (near-exact) b and hn in FP64, rounded once.
__device__ __forceinline__ float dsc_score_d(const Theta* __restrict__ th, double b, double hn) {
  const int nv = th->nv;
  double r = -INFINITY;
#pragma unroll
  for (int v = 1; v < DSC_MAXV; ++v) {
    if (v < nv) {
      const double ph = (double)th->phi[v];
      r = fmax(r, (th->csd[v] + ph * b) - (ph * ph) * hn);
    }
  }
  return (float)r;
}

// Bound on |computed score - real score| given the bound kappa ||y|| ||P_h||
// on the projection error of b: the score is Lipschitz in b with constant
// max |phi_v| (1 for BSC/TSC/MCA), plus the FP32 roundings of the score's
// own arithmetic (about 2 units of 2^-24 of its terms for b - hn, 4 for the
// DSC form with its constant, product and square).
__device__ __forceinline__ float select_delta(int smode, const Theta* __restrict__ th,
                                              float kappa, float ynorm, float pn) {
  if (smode == SCORE_DSC) {
    const float pm = th->phimax;
    return pm * kappa * ynorm * pn + 2.4e-7f * (pm * ynorm * pn + pm * pm * pn * pn + th->csmax);
  }
  return kappa * ynorm * pn + 1.2e-7f * (ynorm * pn + pn * pn);
}

// Exact selection of one point by one wave from its score row (lane l holds
// the latents 64 i + l).  cH and cN are the H'-th and (H'+1)-th largest
// computed scores: given by the caller (have_thr), else found by a radix
// select.  With every computed score within delta of the real one, a latent
// scoring above cH + 2 delta is certainly among the H' best and one below
// cN - 2 delta certainly is not; the latents in between (the band U) are
// re-scored with a compensated dot product (TwoProduct + TwoSum), and the
// missing H' - |C| are taken from U by refined score (ties to the lower
// index).  The point is flagged when the refined H'-th and (H'+1)-th scores
// are within 1e-6 max(1, |r|).
template <int RM>
__device__ __forceinline__ void exact_select_point(const float* __restrict__ brow, int lane, int R, int H, int Hp,
                                   int smode, bool have_thr, float cH, float cN, float delta,
                                   const float* __restrict__ yrow, int D, int Dp,
                                   const float* __restrict__ Pt32,
                                   const float* __restrict__ hn_hi,
                                   const float* __restrict__ hn_lo, int32_t* __restrict__ selp,
                                   float* __restrict__ bcp, uint8_t* flagp,
                                   const Theta* __restrict__ th) {
  float b[RM], sc[RM];
  uint32_t key[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const int h = 64 * i + lane;
    const bool valid = (i < R) && (h < H);
    b[i] = (i < R) ? brow[h] : 0.0f;
    const int hh = h < H ? h : 0;
    float s0;
    if (smode == SCORE_DSC) {
      s0 = dsc_score(th, b[i], hn_hi[hh], hn_lo[hh]);
    } else {
      const float bb = smode == SCORE_ABS ? fabsf(b[i]) : b[i];
      s0 = (bb - hn_hi[hh]) - hn_lo[hh];
    }
    sc[i] = valid ? s0 : 0.0f;
    key[i] = valid ? f2key(sc[i]) : 0u;
  }
  uint64_t selm[RM];
  uint8_t flag = 0;
  if (Hp >= H) {
#pragma unroll
    for (int i = 0; i < RM; ++i) selm[i] = ballot64((i < R) && (64 * i + lane < H));
  } else {
    if (!have_thr) {
      radix_select<RM>(key, R, Hp, selm);
      float mH = INFINITY, mN = -INFINITY;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const bool valid = (i < R) && (64 * i + lane < H);
        if (valid) {
          if ((selm[i] >> lane) & 1ull) mH = fminf(mH, sc[i]);
          else mN = fmaxf(mN, sc[i]);
        }
      }
      cH = wave_min(mH);
      cN = wave_max(mN);
    }
    // decided by the threshold only when even the smallest true gap
    // (computed gap - 2 delta) lies outside the flag band
    const float gap = cH - cN;
    if (!(gap - 2.0f * delta > 1e-6f * fmaxf(1.0f, fabsf(cH) + 2.0f * delta))) {
      const float lo_b = cN - 2.0f * delta, hi_b = cH + 2.0f * delta;
      uint64_t Um[RM], Cm[RM];
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const bool valid = (i < R) && (64 * i + lane < H);
        Um[i] = ballot64(valid && sc[i] >= lo_b && sc[i] <= hi_b);
        Cm[i] = ballot64(valid && sc[i] > hi_b);
      }
      // re-score the band, four latents at a time, 256 depths per round:
      // every load of a round is issued before the first use
      uint64_t rem[RM];
#pragma unroll
      for (int i = 0; i < RM; ++i) rem[i] = Um[i];
      while (true) {
        int hs[4];
        int cnt = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          int h = -1;
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            if (h < 0 && rem[i] != 0ull) {
              h = 64 * i + __ffsll((unsigned long long)rem[i]) - 1;
              rem[i] &= rem[i] - 1ull;
            }
          }
          hs[m] = h;
          cnt += h >= 0 ? 1 : 0;
        }
        if (cnt == 0) break;
        float ss[4] = {0.f, 0.f, 0.f, 0.f}, cc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int d0 = 0; d0 < D; d0 += 256) {
          float yv[4], pv[4][4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int d = d0 + 64 * k + lane;
            const float y = yrow[d < D ? d : D - 1];
            yv[k] = d < D ? y : 0.0f;
          }
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int d = d0 + 64 * k + lane;
              const int hm = hs[m] >= 0 ? hs[m] : hs[0];
              pv[m][k] = Pt32[(int64_t)hm * Dp + (d < D ? d : D - 1)];
            }
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              float pr, e, s2, e2;
              two_prod(yv[k], pv[m][k], pr, e);
              two_sum(ss[m], pr, s2, e2);
              ss[m] = s2;
              cc[m] += e2 + e;
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (m < cnt) {
            float s = ss[m], c = cc[m];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
              const float so = __shfl_xor(s, o, 64), co = __shfl_xor(c, o, 64);
              float s2, e2;
              two_sum(s, so, s2, e2);
              s = s2;
              c = c + co + e2;
            }
            const int h = hs[m];
            float rr;
            if (smode == SCORE_DSC) {
              rr = dsc_score_d(th, (double)s + (double)c, (double)hn_hi[h] + (double)hn_lo[h]);
            } else {
              const float sg = (smode == SCORE_ABS && s < 0.0f) ? -1.0f : 1.0f;
              rr = (sg * s - hn_hi[h]) + (sg * c - hn_lo[h]);
            }
            const int i = h >> 6, l2 = h & 63;
#pragma unroll
            for (int i2 = 0; i2 < RM; ++i2) {
              if (i2 == i && lane == l2) {
                sc[i2] = rr;
                b[i2] = s + c;
                key[i2] = f2key(rr);
              }
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        if (!((Um[i] >> lane) & 1ull)) key[i] = ((Cm[i] >> lane) & 1ull) ? 0xFFFFFFFFu : 0u;
      }
      radix_select<RM>(key, R, Hp, selm);
      float uH = INFINITY, uN = -INFINITY;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        if ((Um[i] >> lane) & 1ull) {
          if ((selm[i] >> lane) & 1ull) uH = fminf(uH, sc[i]);
          else uN = fmaxf(uN, sc[i]);
        }
      }
      uH = wave_min(uH);
      uN = wave_max(uN);
      flag = (uH - uN <= 1e-6f * fmaxf(1.0f, fabsf(uH))) ? 1 : 0;
    } else {
      // the threshold decides
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const bool valid = (i < R) && (64 * i + lane < H);
        selm[i] = ballot64(valid && sc[i] >= cH);
      }
    }
  }
  int base = 0;
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const uint64_t m = selm[i];
    if ((m >> lane) & 1ull) {
      const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
      selp[pos] = 64 * i + lane;
      bcp[pos] = b[i];
    }
    base += __popcll(m);
  }
  if (lane == 0 && flagp) *flagp = flag;
}

}  // namespace prosper
