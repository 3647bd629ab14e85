// Projection and preselection (rows a2 and a3 of the hot path).
//
// For a tile of TM data points one workgroup (4 waves) computes b = P y for
// every latent with MFMA (P = W^T, or max(W,0)^T for max superposition),
// turns b into the ranking score of each latent, and keeps the H' best
// (ties to the lower latent index).  The ranking score is the singleton
// log-joint up to latent-independent terms and the positive factor 1/sigma^2:
//   r_h = b_h - 1/2 ||P_h||^2           (BSC, MCA)
//   r_h = |b_h| - 1/2 ||P_h||^2         (TSC: better of the two signs)
//
// Selection is exact with respect to the real-valued scores: the projection
// error is bounded by delta (the standard FP32 summation bound plus, for the
// BF16 split, the representation error of the head/tail pair), and whenever
// the H'-th and (H'+1)-th computed scores lie within 2 delta the latents in
// that band are re-scored with a compensated FP32 dot product (TwoProduct +
// TwoSum), which leaves only genuine near-ties undecided.  Such points are
// flagged when the refined gap is within 1e-6 max(1, |r|).
//
// MFMA layouts (CDNA wave64, 16x16 output tile, lane l: row/col l%16):
//   v_mfma_f32_16x16x4_f32  : A[l%16][k-group l/16], one k per lane
//   v_mfma_f32_16x16x32_bf16: A[l%16][8 consecutive k of group l/16]
//   C: 4 values per lane at rows 4(l/16)+i, column l%16
// The k index of group q runs over a contiguous quarter of the padded depth
// (k = q Dp/4 + t) so that each lane reads 16 contiguous bytes per step; A
// and B use the same map, so the contraction is unchanged.
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

template <int PREC, int TM, int RM>
__global__ __launch_bounds__(256, 2) void k_project_select(
    const float* __restrict__ Y, int64_t N, int D, int Dp, int H,
    const float* __restrict__ Pt32, const bf16* __restrict__ Pt_hi,
    const bf16* __restrict__ Pt_lo, const float* __restrict__ hn_hi,
    const float* __restrict__ hn_lo, const float* __restrict__ pnorm, int Hp, int score_abs,
    float kappa, int32_t* __restrict__ sel, float* __restrict__ bc, float* __restrict__ yy_out,
    uint8_t* __restrict__ flagged, double* __restrict__ scal) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float yyS[TM];
  __shared__ double yydS[TM];
  constexpr int MT = TM / 16;       // point tiles of 16
  constexpr int GPW = 4 / MT;       // latent groups (of 64) per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t n0 = (int64_t)blockIdx.x * TM;
  const int Hpad = round_up(H, 64);
  const int Hs = Hpad + 4;
  const int ngroups = Hpad / 64;
  const int kq = Dp / 4;

  // ---- stage the Y tile (FP32, or BF16 head/tail) and ||y||^2 in FP64
  if constexpr (PREC == PROSPER_FP32) {
    float* Ys = reinterpret_cast<float*>(smem);
    const int ys = Dp + 4;
    for (int r = wave; r < TM; r += 4) {
      const int64_t n = n0 + r;
      double acc = 0.0;
      for (int d = lane; d < Dp; d += 64) {
        float v = (n < N && d < D) ? Y[n * D + d] : 0.0f;
        Ys[r * ys + d] = v;
        acc = fma((double)v, (double)v, acc);
      }
      acc = wave_sum_d(acc);
      if (lane == 0) {
        yyS[r] = (float)acc;
        yydS[r] = acc;
      }
    }
  } else {
    bf16* Yh = reinterpret_cast<bf16*>(smem);
    const int ys = Dp + 8;
    bf16* Yl = Yh + TM * ys;
    for (int r = wave; r < TM; r += 4) {
      const int64_t n = n0 + r;
      double acc = 0.0;
      for (int d = lane; d < Dp; d += 64) {
        float v = (n < N && d < D) ? Y[n * D + d] : 0.0f;
        bf16 hi = (bf16)v;
        Yh[r * ys + d] = hi;
        Yl[r * ys + d] = (bf16)(v - (float)hi);
        acc = fma((double)v, (double)v, acc);
      }
      acc = wave_sum_d(acc);
      if (lane == 0) {
        yyS[r] = (float)acc;
        yydS[r] = acc;
      }
    }
  }
  __syncthreads();

  // ---- b = P y for the tile: MFMA, FP32 accumulation
  f32x4 acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[s][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int gi = 0; gi < GPW; ++gi) {
    const int g = wave + 4 * gi;
    if (g >= ngroups) break;
    if constexpr (PREC == PROSPER_FP32) {
      const float* Ys = reinterpret_cast<const float*>(smem);
      const int ys = Dp + 4;
      for (int t = 0; t < kq; t += 4) {
        float4 a[MT], b[4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          a[mt] = *reinterpret_cast<const float4*>(&Ys[(mt * 16 + r16) * ys + q * kq + t]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const int h = g * 64 + nt * 16 + r16;
          b[nt] = (h < H) ? *reinterpret_cast<const float4*>(&Pt32[(int64_t)h * Dp + q * kq + t])
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            f32x4& c = acc[gi * MT + mt][nt];
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt].x, b[nt].x, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt].y, b[nt].y, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt].z, b[nt].z, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt].w, b[nt].w, c, 0, 0, 0);
          }
      }
    } else {
      const bf16* Yh = reinterpret_cast<const bf16*>(smem);
      const int ys = Dp + 8;
      const bf16* Yl = Yh + TM * ys;
      for (int t = 0; t < kq; t += 8) {
        bf16x8 ah[MT], al[MT], bh[4], bl[4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int o = (mt * 16 + r16) * ys + q * kq + t;
          ah[mt] = *reinterpret_cast<const bf16x8*>(&Yh[o]);
          al[mt] = *reinterpret_cast<const bf16x8*>(&Yl[o]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const int h = g * 64 + nt * 16 + r16;
          if (h < H) {
            const int64_t o = (int64_t)h * Dp + q * kq + t;
            bh[nt] = *reinterpret_cast<const bf16x8*>(&Pt_hi[o]);
            bl[nt] = *reinterpret_cast<const bf16x8*>(&Pt_lo[o]);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              bh[nt][e] = (bf16)0.0f;
              bl[nt][e] = (bf16)0.0f;
            }
          }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            f32x4& c = acc[gi * MT + mt][nt];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bh[nt], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bl[nt], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh[nt], c, 0, 0, 0);
          }
      }
    }
  }
  __syncthreads();  // the Y tile is dead from here on; Bs reuses its memory

  float* Bs = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int gi = 0; gi < GPW; ++gi) {
    const int g = wave + 4 * gi;
    if (g >= ngroups) break;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          Bs[(mt * 16 + 4 * q + i) * Hs + g * 64 + nt * 16 + r16] = acc[gi * MT + mt][nt][i];
  }
  __syncthreads();

  // ---- per point: scores, exact top-H', outputs (one wave per point)
  const int R = Hpad / 64;
  float hnh[RM], hnl[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const int h = 64 * i + lane;
    hnh[i] = (i < R && h < H) ? hn_hi[h] : 0.0f;
    hnl[i] = (i < R && h < H) ? hn_lo[h] : 0.0f;
  }
  const float pn = *pnorm;

  for (int r = wave; r < TM; r += 4) {
    const int64_t n = n0 + r;
    if (n >= N) break;
    float b[RM], sc[RM];
    uint32_t key[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      const int h = 64 * i + lane;
      const bool valid = (i < R) && (h < H);
      b[i] = (i < R) ? Bs[r * Hs + h] : 0.0f;
      const float bb = score_abs ? fabsf(b[i]) : b[i];
      sc[i] = (bb - hnh[i]) - hnl[i];
      key[i] = valid ? f2key(sc[i]) : 0u;
    }
    uint64_t selm[RM];
    uint8_t flag = 0;
    if (Hp >= H) {
#pragma unroll
      for (int i = 0; i < RM; ++i) selm[i] = ballot64((i < R) && (64 * i + lane < H));
    } else {
      radix_select<RM>(key, R, Hp, selm);
      float cH = INFINITY, cN = -INFINITY;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const bool valid = (i < R) && (64 * i + lane < H);
        if (valid) {
          if ((selm[i] >> lane) & 1ull) cH = fminf(cH, sc[i]);
          else cN = fmaxf(cN, sc[i]);
        }
      }
      cH = wave_min(cH);
      cN = wave_max(cN);
      const float ynorm = sqrtf(yyS[r]);
      const float delta = kappa * ynorm * pn + 1.2e-7f * (ynorm * pn + pn * pn);
      if (!(cH - cN > 2.0f * delta)) {
        // band of undecided latents: re-score with a compensated dot product
        const float lo_b = cH - 2.0f * delta, hi_b = cN + 2.0f * delta;
        uint64_t Um[RM], Cm[RM];
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          const bool valid = (i < R) && (64 * i + lane < H);
          Um[i] = ballot64(valid && sc[i] >= lo_b && sc[i] <= hi_b);
          Cm[i] = ballot64(valid && sc[i] > hi_b);
        }
        const float* yrow = Y + n * D;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          uint64_t m = Um[i];
          while (m) {
            const int l2 = __ffsll((unsigned long long)m) - 1;
            m &= m - 1ull;
            const int h = 64 * i + l2;
            const float* prow = Pt32 + (int64_t)h * Dp;
            float s = 0.0f, c = 0.0f;
            for (int d = lane; d < D; d += 64) {
              float p, e, s2, e2;
              two_prod(yrow[d], prow[d], p, e);
              two_sum(s, p, s2, e2);
              s = s2;
              c += e2 + e;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
              const float so = __shfl_xor(s, o, 64), co = __shfl_xor(c, o, 64);
              float s2, e2;
              two_sum(s, so, s2, e2);
              s = s2;
              c = c + co + e2;
            }
            const float sg = (score_abs && s < 0.0f) ? -1.0f : 1.0f;
            const float rr = (sg * s - hn_hi[h]) + (sg * c - hn_lo[h]);
            if (lane == l2) {
              sc[i] = rr;
              b[i] = s + c;
              key[i] = f2key(rr);
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
      }
    }
    int base = 0;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      const uint64_t m = selm[i];
      if ((m >> lane) & 1ull) {
        const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
        sel[n * Hp + pos] = 64 * i + lane;
        bc[n * Hp + pos] = b[i];
      }
      base += __popcll(m);
    }
    if (lane == 0) {
      yy_out[n] = yyS[r];
      if (flagged) flagged[n] = flag;
    }
  }
  if (scal && threadIdx.x == 0) {  // [2] sum ||y||^2, [4] number of points
    double s = 0.0;
    int cnt = 0;
    for (int r = 0; r < TM && n0 + r < N; ++r, ++cnt) s += yydS[r];
    atomicAdd(&scal[2], s);
    atomicAdd(&scal[4], (double)cnt);
  }
}

template <int PREC, int TM, int RM>
static hipError_t launch_ps(const float* Y, int64_t N, int D, int Dp, int H, int Hp,
                            int score_abs, float kappa, const Prepared& p, const Scratch& s,
                            uint8_t* flagged, double* scal, size_t lds, hipStream_t st) {
  auto kern = k_project_select<PREC, TM, RM>;
  static size_t configured = 0;
  if (lds > configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  const int64_t nblk = (N + TM - 1) / TM;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(256), lds, st, Y, N, D, Dp, H, p.Pt32,
                     p.Pt_hi, p.Pt_lo, p.hn_hi, p.hn_lo, p.pnorm, Hp, score_abs, kappa, s.sel,
                     s.bc, s.yy, flagged, scal);
  return hipGetLastError();
}

// Points per workgroup: the score tile (TM x H) and the Y tile (TM x D) share
// at most ~80 KB of LDS so that two workgroups fit on a CU.
static int choose_tm(int Dp, int H, int prec) {
  const int Hpad = round_up(H, 64);
  int tm = Hpad <= 256 ? 64 : (Hpad <= 512 ? 32 : 16);
  auto bytes = [&](int t) {
    size_t yrow = (prec == PROSPER_FP32) ? (size_t)(Dp + 4) * 4 : (size_t)(Dp + 8) * 4;
    size_t brow = (size_t)(Hpad + 4) * 4;
    return (size_t)t * (yrow > brow ? yrow : brow);
  };
  while (tm > 16 && bytes(tm) > 80 * 1024) tm /= 2;
  return tm;
}

size_t project_lds_bytes(int Dp, int H, int prec, int tm) {
  const int Hpad = round_up(H, 64);
  size_t yrow = (prec == PROSPER_FP32) ? (size_t)(Dp + 4) * 4 : (size_t)(Dp + 8) * 4;
  size_t brow = (size_t)(Hpad + 4) * 4;
  return (size_t)tm * (yrow > brow ? yrow : brow);
}

hipError_t launch_project_select(int model, int prec, const float* Y, int64_t N, int D, int Dp,
                                 int H, int Hp, const Prepared& p, const Scratch& s,
                                 uint8_t* flagged, double* scal, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int score_abs = (model == PROSPER_TSC) ? 1 : 0;
  const double u = 1.0 / 16777216.0;  // 2^-24
  const float kappa = (prec == PROSPER_FP32)
                          ? (float)(2.0 * Dp * u)
                          : (float)(2.0 * (1.0 / 65536.0 + 3.0 * Dp * u));
  const int tm = choose_tm(Dp, H, prec);
  const size_t lds = project_lds_bytes(Dp, H, prec, tm);
  const int Hpad = round_up(H, 64);
  const bool small = Hpad <= 256;
#define PS_CASE(P, T, R) \
  return launch_ps<P, T, R>(Y, N, D, Dp, H, Hp, score_abs, kappa, p, s, flagged, scal, lds, st)
  if (prec == PROSPER_FP32) {
    if (small) {
      if (tm == 64) PS_CASE(PROSPER_FP32, 64, 4);
      if (tm == 32) PS_CASE(PROSPER_FP32, 32, 4);
      PS_CASE(PROSPER_FP32, 16, 4);
    }
    if (tm == 32) PS_CASE(PROSPER_FP32, 32, 16);
    PS_CASE(PROSPER_FP32, 16, 16);
  } else {
    if (small) {
      if (tm == 64) PS_CASE(PROSPER_BF16, 64, 4);
      if (tm == 32) PS_CASE(PROSPER_BF16, 32, 4);
      PS_CASE(PROSPER_BF16, 16, 4);
    }
    if (tm == 32) PS_CASE(PROSPER_BF16, 32, 16);
    PS_CASE(PROSPER_BF16, 16, 16);
  }
#undef PS_CASE
}

}  // namespace prosper
