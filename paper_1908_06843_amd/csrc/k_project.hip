// Projection and preselection (rows a2 and a3 of the hot path).
//
// For a tile of TM data points one workgroup (4 waves) computes b = P y for
// every latent with MFMA (P = W^T, or max(W,0)^T for max superposition),
// turns b into the ranking score of each latent, and keeps the H' best
// (ties to the lower latent index).  The ranking score is the singleton
// log-joint up to latent-independent terms and the positive factor 1/sigma^2:
//   r_h = b_h - 1/2 ||P_h||^2           (BSC, MCA)
//   r_h = |b_h| - 1/2 ||P_h||^2         (TSC: better of the two signs)
//   r_h = max_v cs_v + phi_v b_h - phi_v^2 1/2 ||P_h||^2   (DSC: best value)
// (score modes of k_select.hpp; the error bound delta of each in select_delta)
//
// Selection is exact with respect to the real-valued scores: the projection
// error is bounded by delta (the FP32 summation bound plus, for the BF16
// split, the representation error of the head/tail pair).  A point whose
// H'-th and (H'+1)-th computed scores are further apart than 2 delta is
// decided by the computed scores; otherwise the latents in the undecided
// band are re-scored with a compensated FP32 dot product (TwoProduct +
// TwoSum), which leaves only genuine near-ties, flagged when the refined gap
// is within 1e-6 max(1, |r|).
//
// MFMA layouts (CDNA wave64, 16x16 output tile, lane l: row/col l%16):
//   v_mfma_f32_16x16x4_f32  : A[l%16][k-group l/16], one k per lane
//   v_mfma_f32_16x16x32_bf16: A[l%16][8 consecutive k of group l/16]
//   C: 4 values per lane at rows 4(l/16)+i, column l%16
// Within each block of 64 depths, lane group q owns depths 16 q .. 16 q + 15
// (spread over the block's MFMAs), so the four groups of a row read one
// whole cache line of P per block; A and B use the same map, so the
// contraction is unchanged.
#include <algorithm>

#include "dev_common.hpp"
#include "k_select.hpp"
#include "prosper_internal.hpp"

namespace prosper {

// Selection lists of the lane-per-point pass (H' <= FAST_HP).
static constexpr int FAST_HP = 12;
static constexpr int FAST_KL = FAST_HP + 1;

template <int TM>
struct SelLds {
  union {
    float lists[3][FAST_KL][TM];    // per-quarter running lists of waves 1..3
    uint16_t qsel[4][TM][FAST_HP];  // selected latents found by each quarter
  } u;
  uint8_t qcnt[4][TM];
  float thr[TM];
  float thrN[TM];
  uint8_t fast[TM];
  uint8_t slow[TM];
  int nslow;
  int dbase;
};

// One workgroup (4 waves) per tile of TM points:
//   1. Y tile -> LDS (FP32, or BF16 head/tail), ||y||^2 in FP64;
//   2. b = P y by MFMA, the next B fragments prefetched during each step;
//   3. b -> LDS score tile (row per point, odd stride);
//   4. FAST (H' <= 12 < H): every lane takes one point; wave w keeps the
//      H'+1 largest scores of latent quarter w, wave 0 merges the four lists.
//      A point whose H'-th and (H'+1)-th scores are further apart than the
//      error bound 2 delta plus the flag distance is decided by threshold:
//      its selection is every latent scoring at least the H'-th value.  The
//      remaining points go through the exact per-wave path above: in
//      k_select_deferred when the caller gives a deferral list with room
//      (the b row and the thresholds are written out), else here.
//      Without FAST every point takes the exact path here.
// Ranking score of latent h in the lane-per-point pass: the BSC/TSC/MCA
// forms as written there, or the DSC score of k_select.hpp.
template <bool DSC>
__device__ __forceinline__ float fast_score(float bv, int score_abs, float hh, float hl,
                                            const Theta* __restrict__ th) {
  if constexpr (DSC) {
    return dsc_score(th, bv, hh, hl);
  } else {
    const float bb = score_abs ? fabsf(bv) : bv;
    return (bb - hh) - hl;
  }
}

template <int PREC, int TM, int RM, bool FAST, bool DSC = false>
__global__ __launch_bounds__(256, 2) void k_project_select(
    const float* __restrict__ Y, int64_t N, int D, int Dp, int H,
    const float* __restrict__ Pt32, const bf16* __restrict__ Pt_hi,
    const bf16* __restrict__ Pt_lo, const float* __restrict__ hn_hi,
    const float* __restrict__ hn_lo, const float* __restrict__ pnorm, int Hp, int score_abs,
    float kappa, int32_t* __restrict__ sel, float* __restrict__ bc, float* __restrict__ yy_out,
    uint8_t* __restrict__ flagged, double* __restrict__ scal, int tile_bytes,
    float* __restrict__ defer, int defer_cap, int32_t* __restrict__ defer_count,
    const Theta* __restrict__ th) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float yyS[TM];
  __shared__ double yydS[TM];
  __shared__ SelLds<TM> sl;
  constexpr int MT = TM / 16;       // point tiles of 16
  constexpr int GPW = 4 / MT;       // latent groups (of 64) per wave
  constexpr int RPW = TM / 4;       // staged rows per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t n0 = (int64_t)blockIdx.x * TM;
  const int Hpad = round_up(H, 64);
  const int Hs = Hpad + 1;
  const int ngroups = Hpad / 64;
  // 1/2 ||P_h||^2 (head, tail) of every latent, behind the tile in LDS
  float* hnS = reinterpret_cast<float*>(smem + tile_bytes);
  for (int h = threadIdx.x; h < Hpad; h += 256) {
    hnS[h] = h < H ? hn_hi[h] : 0.0f;
    hnS[Hpad + h] = h < H ? hn_lo[h] : 0.0f;
  }

  // ---- 1. stage the Y tile: every load of a lane issued before any use
  {
    const int nc4 = Dp >> 2;            // float4 per padded row
    const int cj = (nc4 + 63) >> 6;     // per lane and row (<= 4)
    const bool vec = (D & 3) == 0;
    double part[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) part[rr] = 0.0;
    for (int j = 0; j < cj; ++j) {
      const int c4 = lane + 64 * j;
      // unconditional loads from clamped addresses (masked afterwards), so
      // that the RPW loads of a lane are all in flight together
      float4 v[RPW];
      if (vec) {
        const bool cok = 4 * c4 < D;
        const int cc = cok ? 4 * c4 : 0;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
          const int64_t n = n0 + wave * RPW + rr;
          const int64_t nn = n < N ? n : N - 1;
          const float4 x = *reinterpret_cast<const float4*>(Y + nn * D + cc);
          v[rr] = (cok && n < N) ? x : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      } else {
        const int d = 4 * c4;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
          const int64_t n = n0 + wave * RPW + rr;
          const bool nok = n < N;
          const float* yr = Y + (nok ? n : N - 1) * D;
          float e[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float x = yr[min(d + k, D - 1)];
            e[k] = (nok && d + k < D) ? x : 0.f;
          }
          v[rr] = make_float4(e[0], e[1], e[2], e[3]);
        }
      }
      if (c4 < nc4) {
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
          const int r = wave * RPW + rr;
          const float4 x = v[rr];
          if constexpr (PREC == PROSPER_FP32) {
            float* Ys = reinterpret_cast<float*>(smem);
            *reinterpret_cast<float4*>(&Ys[r * (Dp + 4) + 4 * c4]) = x;
          } else {
            bf16* Yh = reinterpret_cast<bf16*>(smem);
            bf16* Yl = Yh + TM * (Dp + 8);
            typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
            bf16x4 hi, lo;
            hi[0] = (bf16)x.x;
            hi[1] = (bf16)x.y;
            hi[2] = (bf16)x.z;
            hi[3] = (bf16)x.w;
            *reinterpret_cast<bf16x4*>(&Yh[r * (Dp + 8) + 4 * c4]) = hi;
            if constexpr (PREC == PROSPER_BF16) {
              lo[0] = (bf16)(x.x - (float)hi[0]);
              lo[1] = (bf16)(x.y - (float)hi[1]);
              lo[2] = (bf16)(x.z - (float)hi[2]);
              lo[3] = (bf16)(x.w - (float)hi[3]);
              *reinterpret_cast<bf16x4*>(&Yl[r * (Dp + 8) + 4 * c4]) = lo;
            }
          }
          double a = part[rr];
          a = fma((double)x.x, (double)x.x, a);
          a = fma((double)x.y, (double)x.y, a);
          a = fma((double)x.z, (double)x.z, a);
          a = fma((double)x.w, (double)x.w, a);
          part[rr] = a;
        }
      }
    }
    double tot;
    const int rr = wave_sum_rows<RPW>(part, lane, tot);
    if ((lane & (64 / RPW - 1)) == 0) {
      yyS[wave * RPW + rr] = (float)tot;
      yydS[wave * RPW + rr] = tot;
    }
  }
  __syncthreads();

  // ---- 2. b = P y for the tile: MFMA, FP32 accumulation
  // BF16: head*head products in acc, the two cross products in accx (kept
  // apart so that the accumulation error of each is relative to its own
  // magnitude); FP32 and the single BF16 product (BF16X1) use acc only
  constexpr int NX = (PREC == PROSPER_BF16) ? 4 : 1;
  f32x4 acc[4][4], accx[NX][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[s][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NX; ++s)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) accx[s][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int gi = 0; gi < GPW; ++gi) {
    const int g = wave + 4 * gi;
    if (g >= ngroups) break;
    // B rows of this lane (clamped inside P; rows >= H are zeroed)
    int64_t boff[4];
    bool bval[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int h = g * 64 + nt * 16 + r16;
      bval[nt] = h < H;
      boff[nt] = (int64_t)(h < H ? h : H - 1) * Dp + 16 * q;
    }
    // k order inside a block of 64 depths: lane group q owns the 16
    // consecutive depths [16 q, 16 q + 16), so the four groups of a row read
    // one whole 128-byte line of P per block; A fragments use the same order.
    if constexpr (PREC == PROSPER_FP32) {
      // 16x16x4 FP32: MFMA m (0..15) of a block takes depth 16 q + m of lane group q
      const float* Ys = reinterpret_cast<const float*>(smem);
      const int ys = Dp + 4;
      float4 b[4][4], bn[4][4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          b[nt][v] = *reinterpret_cast<const float4*>(&Pt32[boff[nt] + 4 * v]);
      for (int t = 0; t < Dp; t += 64) {
        const int tn = (t + 64 < Dp) ? t + 64 : t;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            bn[nt][v] = *reinterpret_cast<const float4*>(&Pt32[boff[nt] + tn + 4 * v]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!bval[nt]) b[nt][v] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          float4 a[4];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            a[v] = *reinterpret_cast<const float4*>(&Ys[(mt * 16 + r16) * ys + t + 16 * q + 4 * v]);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            f32x4& c = acc[gi * MT + mt][nt];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[v].x, b[nt][v].x, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[v].y, b[nt][v].y, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[v].z, b[nt][v].z, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[v].w, b[nt][v].w, c, 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) b[nt][v] = bn[nt][v];
      }
    } else {
      // 16x16x32 BF16: MFMA j (0, 1) of a block takes depths 16 q + 8 j .. + 8
      // (BF16X1: the head*head product only)
      constexpr bool SPLIT = PREC == PROSPER_BF16;
      const bf16* Yh = reinterpret_cast<const bf16*>(smem);
      const int ys = Dp + 8;
      const bf16* Yl = Yh + TM * ys;
      typedef __attribute__((ext_vector_type(4))) int i32x4;
      i32x4 bh[4][2], bl[4][2], bhn[4][2], bln[4][2];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          bh[nt][j] = *reinterpret_cast<const i32x4*>(&Pt_hi[boff[nt] + 8 * j]);
          if constexpr (SPLIT) bl[nt][j] = *reinterpret_cast<const i32x4*>(&Pt_lo[boff[nt] + 8 * j]);
        }
      for (int t = 0; t < Dp; t += 64) {
        const int tn = (t + 64 < Dp) ? t + 64 : t;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            bhn[nt][j] = *reinterpret_cast<const i32x4*>(&Pt_hi[boff[nt] + tn + 8 * j]);
            if constexpr (SPLIT)
              bln[nt][j] = *reinterpret_cast<const i32x4*>(&Pt_lo[boff[nt] + tn + 8 * j]);
          }
        const i32x4 zero = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          bf16x8 ah[MT], al[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int o = (mt * 16 + r16) * ys + t + 16 * q + 8 * j;
            ah[mt] = *reinterpret_cast<const bf16x8*>(&Yh[o]);
            if constexpr (SPLIT) al[mt] = *reinterpret_cast<const bf16x8*>(&Yl[o]);
          }
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 bhv = __builtin_bit_cast(bf16x8, bval[nt] ? bh[nt][j] : zero);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              f32x4& c = acc[gi * MT + mt][nt];
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bhv, c, 0, 0, 0);
              if constexpr (SPLIT) {
                const bf16x8 blv = __builtin_bit_cast(bf16x8, bval[nt] ? bl[nt][j] : zero);
                f32x4& cx = accx[(gi * MT + mt) % NX][nt];
                cx = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], blv, cx, 0, 0, 0);
                cx = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bhv, cx, 0, 0, 0);
              }
            }
          }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            bh[nt][j] = bhn[nt][j];
            if constexpr (SPLIT) bl[nt][j] = bln[nt][j];
          }
      }
    }
  }
  __syncthreads();  // the Y tile is dead from here on; Bs reuses its memory

  // ---- 3. scores tile
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
          Bs[(mt * 16 + 4 * q + i) * Hs + g * 64 + nt * 16 + r16] =
              (PREC == PROSPER_BF16) ? acc[gi * MT + mt][nt][i] + accx[(gi * MT + mt) % NX][nt][i]
                                     : acc[gi * MT + mt][nt][i];
  }
  __syncthreads();

  const int R = Hpad / 64;
  const float pn = *pnorm;
  if constexpr (FAST) {
    // ---- 4a. per-quarter running lists (lane = point)
    const int Q = Hpad / 4;
    const int hq0 = wave * Q;
    const int hq1 = min(hq0 + Q, H);
    const int p = lane;
    const bool plane = p < TM;
    const float* brow = Bs + (plane ? p : 0) * Hs;
    float tl[FAST_KL];
#pragma unroll
    for (int k = 0; k < FAST_KL; ++k) tl[k] = -INFINITY;
#pragma unroll 8
    for (int h = hq0; h < hq1; ++h) {
      const float bv = brow[h];
      list_insert<FAST_KL>(tl, fast_score<DSC>(bv, score_abs, hnS[h], hnS[Hpad + h], th));
    }
    if (wave > 0 && plane) {
#pragma unroll
      for (int k = 0; k < FAST_KL; ++k) sl.u.lists[wave - 1][k][p] = tl[k];
    }
    __syncthreads();
    // ---- 4b. merge, threshold, fast / exact decision
    if (wave == 0) {
      if (plane) {
        for (int w2 = 0; w2 < 3; ++w2)
          for (int k = 0; k <= Hp; ++k) list_insert<FAST_KL>(tl, sl.u.lists[w2][k][p]);
      }
      const int64_t n = n0 + p;
      const bool valid = plane && n < N;
      const float cH = list_at<FAST_KL>(tl, Hp - 1), cN = list_at<FAST_KL>(tl, Hp);
      const float ynorm = sqrtf(valid ? yyS[p] : 0.0f);
      const float delta = select_delta(score_abs, th, kappa, ynorm, pn);
      const float gap = cH - cN;
      const bool fast =
          valid && gap - 2.0f * delta > 1e-6f * fmaxf(1.0f, fabsf(cH) + 2.0f * delta);
      const uint64_t slowm = ballot64(valid && !fast);
      if (plane) {
        sl.thr[p] = cH;
        sl.thrN[p] = cN;
        sl.fast[p] = fast ? 1 : 0;
        if (valid && !fast) sl.slow[__popcll(slowm & ((1ull << lane) - 1ull))] = (uint8_t)p;
      }
      if (lane == 0) sl.nslow = __popcll(slowm);
    }
    __syncthreads();
    // ---- 4c. each quarter lists its latents at or above the threshold
    if (plane) {
      const bool f = sl.fast[p] != 0;
      const float thr = sl.thr[p];
      int cnt = 0;
#pragma unroll 8
      for (int h = hq0; h < hq1; ++h) {
        const float v = fast_score<DSC>(brow[h], score_abs, hnS[h], hnS[Hpad + h], th);
        if (f && v >= thr && cnt < FAST_HP) {
          sl.u.qsel[wave][p][cnt] = (uint16_t)h;
          ++cnt;
        }
      }
      sl.qcnt[wave][p] = (uint8_t)cnt;
    }
    __syncthreads();
    // ---- 4d. outputs of the threshold-decided points (coalesced tile rows)
    for (int e = threadIdx.x; e < TM * Hp; e += 256) {
      const int pp = e / Hp, pos = e - pp * Hp;
      const int64_t n = n0 + pp;
      if (n < N && sl.fast[pp]) {
        int rem = pos, w = 0;
        while (w < 3 && rem >= sl.qcnt[w][pp]) {
          rem -= sl.qcnt[w][pp];
          ++w;
        }
        const int h = sl.u.qsel[w][pp][rem < FAST_HP ? rem : FAST_HP - 1];
        sel[n * Hp + pos] = h;
        bc[n * Hp + pos] = Bs[pp * Hs + h];
      }
    }
    if (threadIdx.x < TM) {
      const int64_t n = n0 + threadIdx.x;
      if (n < N && sl.fast[threadIdx.x]) {
        yy_out[n] = yyS[threadIdx.x];
        if (flagged) flagged[n] = 0;
      }
    }
    // ---- 4e. the exact path for the rest: the first nd of them (those that
    // find a free slot in the deferral list) are written out for
    // k_select_deferred, the others are selected here
    const int ns = sl.nslow;
    int nd = 0;
    if (defer_cap > 0 && ns > 0) {
      if (threadIdx.x == 0) sl.dbase = atomicAdd(defer_count, ns);
      __syncthreads();
      const int dbase = sl.dbase;
      nd = dbase < defer_cap ? min(ns, defer_cap - dbase) : 0;
      const int Hrow = Hpad + 8;
      for (int i = wave; i < nd; i += 4) {
        const int r = sl.slow[i];
        const int64_t n = n0 + r;
        float* ent = defer + (int64_t)(dbase + i) * Hrow;
        const float ynorm = sqrtf(yyS[r]);
        const float delta = select_delta(score_abs, th, kappa, ynorm, pn);
        for (int h = lane; h < Hpad; h += 64) ent[8 + h] = Bs[r * Hs + h];
        if (lane == 0) {
          *reinterpret_cast<int64_t*>(ent) = n;
          ent[2] = sl.thr[r];
          ent[3] = sl.thrN[r];
          ent[4] = delta;
          yy_out[n] = yyS[r];
        }
      }
    }
    for (int i = nd + wave; i < ns; i += 4) {
      const int r = sl.slow[i];
      const int64_t n = n0 + r;
      const float ynorm = sqrtf(yyS[r]);
      const float delta = select_delta(score_abs, th, kappa, ynorm, pn);
      exact_select_point<RM>(Bs + r * Hs, lane, R, H, Hp, score_abs, true, sl.thr[r],
                             sl.thrN[r], delta, Y + n * D, D, Dp, Pt32, hn_hi, hn_lo,
                             sel + n * Hp, bc + n * Hp, flagged ? flagged + n : nullptr, th);
      if (lane == 0) yy_out[n] = yyS[r];
    }
  } else {
    for (int r = wave; r < TM; r += 4) {
      const int64_t n = n0 + r;
      if (n >= N) break;
      const float ynorm = sqrtf(yyS[r]);
      const float delta = select_delta(score_abs, th, kappa, ynorm, pn);
      exact_select_point<RM>(Bs + r * Hs, lane, R, H, Hp, score_abs, false, 0.0f, 0.0f, delta,
                             Y + n * D, D, Dp, Pt32, hn_hi, hn_lo, sel + n * Hp, bc + n * Hp,
                             flagged ? flagged + n : nullptr, th);
      if (lane == 0) yy_out[n] = yyS[r];
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

// The exact selection of the points the projection kernel deferred, one wave
// per point over a grid-stride loop (no LDS, so many waves per SIMD hide the
// latency of the band re-scoring).  Entry i < min(count, cap) holds the
// point index, its H'-th and (H'+1)-th computed scores, delta and its b row.
template <int RM>
__global__ __launch_bounds__(256) void k_select_deferred(
    const float* __restrict__ defer, int defer_cap, const int32_t* __restrict__ defer_count,
    const float* __restrict__ Y, int D, int Dp, int H, int Hp, const float* __restrict__ Pt32,
    const float* __restrict__ hn_hi, const float* __restrict__ hn_lo, int score_abs,
    int32_t* __restrict__ sel, float* __restrict__ bc, uint8_t* __restrict__ flagged,
    const Theta* __restrict__ th) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cnt = min(*defer_count, defer_cap);
  const int Hpad = round_up(H, 64);
  const int R = Hpad / 64;
  const int Hrow = Hpad + 8;
  for (int i = blockIdx.x * 4 + wave; i < cnt; i += gridDim.x * 4) {
    const float* ent = defer + (int64_t)i * Hrow;
    const int64_t n = *reinterpret_cast<const int64_t*>(ent);
    exact_select_point<RM>(ent + 8, lane, R, H, Hp, score_abs, true, ent[2], ent[3], ent[4],
                           Y + n * D, D, Dp, Pt32, hn_hi, hn_lo, sel + n * Hp, bc + n * Hp,
                           flagged ? flagged + n : nullptr, th);
  }
}

// The FP32 fix-up of the single-product form (BF16X1): b of every selected
// candidate recomputed from y and the FP32 projection row, so that the state
// walk starts from FP32-accurate b.  One wave per point; each lane holds up
// to 16 depths of y in registers and sums its products with one rounding per
// fused multiply-add before a butterfly sum over the wave.
__global__ __launch_bounds__(256) void k_fixup_bc(const float* __restrict__ Y, int64_t N, int D,
                                                  int Dp, const float* __restrict__ Pt32,
                                                  const int32_t* __restrict__ sel,
                                                  float* __restrict__ bc, int Hp) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nd = (D + 63) >> 6;  // <= 16 (D <= 1024)
  for (int64_t n = (int64_t)blockIdx.x * 4 + wave; n < N; n += (int64_t)gridDim.x * 4) {
    float y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int d = 64 * k + lane;
      y[k] = (k < nd && d < D) ? Y[n * D + d] : 0.0f;
    }
    for (int j = 0; j < Hp; ++j) {
      const int64_t row = (int64_t)sel[n * Hp + j] * Dp;
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int d = 64 * k + lane;
        if (k < nd && d < D) a = __builtin_fmaf(y[k], Pt32[row + d], a);
      }
      a = wave_sum(a);
      if (lane == 0) bc[n * Hp + j] = a;
    }
  }
}

template <int PREC, int TM, int RM, bool FAST, bool DSC = false>
static hipError_t launch_ps(const float* Y, int64_t N, int D, int Dp, int H, int Hp,
                            int score_abs, float kappa, const Prepared& p, const Scratch& s,
                            uint8_t* flagged, double* scal, size_t lds, hipStream_t st) {
  auto kern = k_project_select<PREC, TM, RM, FAST, DSC>;
  hipError_t e0 = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
  if (e0 != hipSuccess) return e0;
  const int64_t nblk = (N + TM - 1) / TM;
  const int tile_bytes = (int)(lds - (size_t)round_up(H, 64) * 8);
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(256), lds, st, Y, N, D, Dp, H, p.Pt32,
                     p.Pt_hi, p.Pt_lo, p.hn_hi, p.hn_lo, p.pnorm, Hp, score_abs, kappa, s.sel,
                     s.bc, s.yy, flagged, scal, tile_bytes, s.defer, FAST ? s.defer_cap : 0,
                     s.defer_count, p.theta);
  if (FAST && s.defer_cap > 0) {
    // at most one wave per entry; 1024 workgroups are what stays resident at
    // this kernel's register count (4 waves per SIMD)
    const int nwg = (int)std::min<int64_t>(1024, ((int64_t)s.defer_cap + 3) / 4);
    hipLaunchKernelGGL(k_select_deferred<RM>, dim3((unsigned)nwg), dim3(256), 0, st, s.defer,
                       s.defer_cap, s.defer_count, Y, D, Dp, H, Hp, p.Pt32, p.hn_hi, p.hn_lo,
                       score_abs, s.sel, s.bc, flagged, p.theta);
  }
  return hipGetLastError();
}

// Dynamic LDS: the score tile (TM x (Hpad + 1)) and the Y tile share one
// region, followed by the half norms of the latents.
size_t project_lds_bytes(int Dp, int H, int prec, int tm) {
  const int Hpad = round_up(H, 64);
  size_t yrow = (prec == PROSPER_FP32) ? (size_t)(Dp + 4) * 4 : (size_t)(Dp + 8) * 4;
  size_t brow = (size_t)(Hpad + 1) * 4;
  return round_up((int)((size_t)tm * (yrow > brow ? yrow : brow)), 16) + (size_t)Hpad * 8;
}

static size_t static_lds_bytes(int tm) {
  const size_t sel = tm == 64 ? sizeof(SelLds<64>) : (tm == 32 ? sizeof(SelLds<32>) : sizeof(SelLds<16>));
  return sel + (size_t)tm * 12 + 64;
}

// Two workgroups per CU: dynamic + static LDS of one within 80 KB.
static int choose_tm(int Dp, int H, int prec) {
  const int Hpad = round_up(H, 64);
  int tm = Hpad <= 256 ? 64 : (Hpad <= 512 ? 32 : 16);
  while (tm > 16 && project_lds_bytes(Dp, H, prec, tm) + static_lds_bytes(tm) > 80 * 1024)
    tm /= 2;
  return tm;
}

int project_defer_capacity(int64_t N, int H, int Hp, int prec) {
  if (!(Hp <= FAST_HP && Hp < H) || N <= 0) return 0;
  // the single-product form's wide band sends most points to the exact path
  const int64_t want = prec == PROSPER_BF16X1 ? N : N / 4 + 1024;
  return (int)std::min<int64_t>(std::min<int64_t>(N, want), 1 << 24);
}

static hipError_t launch_project_select_body(int model, int prec, const float* Y, int64_t N,
                                             int D, int Dp, int H, int Hp, const Prepared& p,
                                             const Scratch& s, uint8_t* flagged, double* scal,
                                             hipStream_t st);

hipError_t launch_project_select(int model, int prec, const float* Y, int64_t N, int D, int Dp,
                                 int H, int Hp, const Prepared& p, const Scratch& s,
                                 uint8_t* flagged, double* scal, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipError_t e = launch_project_select_body(model, prec, Y, N, D, Dp, H, Hp, p, s, flagged, scal, st);
  if (e != hipSuccess || prec != PROSPER_BF16X1) return e;
  const int64_t nwg = std::min<int64_t>((N + 3) / 4, 2048);
  hipLaunchKernelGGL(k_fixup_bc, dim3((unsigned)nwg), dim3(256), 0, st, Y, N, D, Dp, p.Pt32, s.sel,
                     s.bc, Hp);
  return hipGetLastError();
}

static hipError_t launch_project_select_body(int model, int prec, const float* Y, int64_t N,
                                             int D, int Dp, int H, int Hp, const Prepared& p,
                                             const Scratch& s, uint8_t* flagged, double* scal,
                                             hipStream_t st) {
  const int score_abs =
      (model == PROSPER_TSC) ? SCORE_ABS : (model == PROSPER_DSC ? SCORE_DSC : SCORE_LIN);
  // Bound on |computed b - exact b| per unit of ||y|| ||P_h|| (Cauchy-Schwarz
  // on sum |y_d P_hd|).  FP32: every product rounded once, at most D + 1
  // roundings along the FP32 accumulation (padding adds exact zeros).  BF16
  // head/tail split: the dropped tail*tail and the two split remainders are
  // each at most 2^-16 |y_d P_hd|; head*head, head*tail and tail*head are
  // exact in FP32; the head*head sum sees D + 1 roundings, the cross sum
  // (terms below 2^-7 of the head*head ones) 2 D + 1, and one rounding adds
  // the two.  3% slack.
  // BF16X1 (one head*head product): BF16 keeps 8 significant bits, so each
  // operand's head is within 2^-8 of it and a product of heads (exact in
  // FP32) is within 2^-7 + 2^-16 of y_d P_hd, plus the D + 1 roundings of the
  // accumulation.
  const double u = 1.0 / 16777216.0;  // 2^-24
  const float kappa =
      (prec == PROSPER_FP32)
          ? (float)(1.01 * (D + 2) * u)
          : (prec == PROSPER_BF16X1)
                ? (float)(1.03 * (1.0 / 128.0 + 1.0 / 65536.0 + (D + 2) * u))
                : (float)(1.03 * (3.0 / 65536.0 + (D + 2) * u + (2.0 * D + 1) * u / 128.0 + u));
  const int tm = choose_tm(Dp, H, prec);
  const size_t lds = project_lds_bytes(Dp, H, prec, tm);
  const int Hpad = round_up(H, 64);
  const bool small = Hpad <= 256;
  const bool fast = Hp <= FAST_HP && Hp < H;
  // DSC: its own lane-per-point pass for H <= 256 (the exact path otherwise)
  const bool dsc = model == PROSPER_DSC;
  if (dsc && fast && small) {
#define PS_DSC(P, T)                                                                        \
  return launch_ps<P, T, 4, true, true>(Y, N, D, Dp, H, Hp, score_abs, kappa, p, s, flagged, \
                                        scal, lds, st)
    if (prec == PROSPER_FP32) {
      if (tm == 64) PS_DSC(PROSPER_FP32, 64);
      if (tm == 32) PS_DSC(PROSPER_FP32, 32);
      PS_DSC(PROSPER_FP32, 16);
    }
    if (prec == PROSPER_BF16) {
      if (tm == 64) PS_DSC(PROSPER_BF16, 64);
      if (tm == 32) PS_DSC(PROSPER_BF16, 32);
      PS_DSC(PROSPER_BF16, 16);
    }
#undef PS_DSC
  }
#define PS_CASE(P, T, R)                                                                       \
  return (fast && !dsc)                                                                        \
             ? launch_ps<P, T, R, true>(Y, N, D, Dp, H, Hp, score_abs, kappa, p, s, flagged,   \
                                        scal, lds, st)                                         \
             : launch_ps<P, T, R, false>(Y, N, D, Dp, H, Hp, score_abs, kappa, p, s, flagged,  \
                                         scal, lds, st)
  if (prec == PROSPER_FP32) {
    if (small) {
      if (tm == 64) PS_CASE(PROSPER_FP32, 64, 4);
      if (tm == 32) PS_CASE(PROSPER_FP32, 32, 4);
      PS_CASE(PROSPER_FP32, 16, 4);
    }
    if (tm == 32) PS_CASE(PROSPER_FP32, 32, 16);
    PS_CASE(PROSPER_FP32, 16, 16);
  } else if (prec == PROSPER_BF16) {
    if (small) {
      if (tm == 64) PS_CASE(PROSPER_BF16, 64, 4);
      if (tm == 32) PS_CASE(PROSPER_BF16, 32, 4);
      PS_CASE(PROSPER_BF16, 16, 4);
    }
    if (tm == 32) PS_CASE(PROSPER_BF16, 32, 16);
    PS_CASE(PROSPER_BF16, 16, 16);
  } else {
    if (small) {
      if (tm == 64) PS_CASE(PROSPER_BF16X1, 64, 4);
      if (tm == 32) PS_CASE(PROSPER_BF16X1, 32, 4);
      PS_CASE(PROSPER_BF16X1, 16, 4);
    }
    if (tm == 32) PS_CASE(PROSPER_BF16X1, 32, 16);
    PS_CASE(PROSPER_BF16X1, 16, 16);
  }
#undef PS_CASE
}

}  // namespace prosper
