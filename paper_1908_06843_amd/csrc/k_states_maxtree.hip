// Compile-time unrolled state walk for max superposition (MCA, MMCA): rows
// a4-a8 of the hot path for the shapes instantiated below.
//
// Same quantities as the table-driven walk of k_states_max.hip (Eq. 1 + Eq. 2
// with the direct residual for MCA, the residual relative to the zero state
// for MMCA, the hard-max responsibilities for the M-step), organised for
// throughput:
//  * 16 lanes per data point, 4 points per wave, lane l owning pixels
//    l, l + 16, ... (NPIX of them); the H' candidate columns of P and the
//    pixels of y sit in registers;
//  * the states are enumerated at compile time in the canonical table order
//    (number of actives ascending, then lexicographic slot tuples), so every
//    slot index is a constant and the superposition of a state follows from
//    its prefix's by one max per pixel;
//  * per state every lane holds the partial residual over its pixels; a
//    butterfly reduce-scatter over 16 states at a time (DPP within each row
//    of 16 lanes) leaves the full sum of state 16 b + l in lane l, which
//    keeps that state's log-joint and residual in register b;
//  * responsibilities: a second walk over the subset tree decides per pixel
//    which slot of a state attains the maximum (the lower slot on ties) and
//    adds q(s) to that slot's register accumulator, q(s) broadcast from its
//    owner lane by DPP.  Childless states whose posterior weight is below
//    2^-40 of the largest at every point of the wave are skipped: their total
//    contribution to any responsibility is below |K| 2^-40, far under the
//    FP32 rounding of the sums they would enter;
//  * the per-point responsibilities are summed per workgroup in LDS (one
//    workgroup per CU holding A and B of the latents that fit, transposed)
//    with FP32 LDS atomics; the workgroup sums are written out once and a
//    second kernel adds them in FP64.  Latents beyond what LDS holds go
//    through global float atomics.  (Exact fixed-point sums with integer
//    LDS atomics run faster but lose the relative precision of the small
//    sums that the M-step divides; a lock-ordered FP32 read-modify-write
//    ran slower than the atomics.)
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {
namespace {

constexpr int binom_c(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}
constexpr int popc_c(unsigned m) {
  int c = 0;
  for (; m; m &= m - 1u) ++c;
  return c;
}
constexpr int nstates_c(int hp, int g) {
  int s = 0;
  for (int k = 0; k <= g; ++k) s += binom_c(hp, k);
  return s;
}
// Position of a slot set in the canonical table order.
constexpr int canon_c(int hp, unsigned mask) {
  const int k = popc_c(mask);
  int off = 0;
  for (int t = 0; t < k; ++t) off += binom_c(hp, t);
  int r = 0, prev = -1, i = 0;
  for (int a = 0; a < hp; ++a) {
    if ((mask >> a) & 1u) {
      for (int x = prev + 1; x < a; ++x) r += binom_c(hp - 1 - x, k - 1 - i);
      prev = a;
      ++i;
    }
  }
  return off + r;
}

// Lane permutations inside each row of 16 lanes.  Partners of the four
// butterfly stages: l^15 (row mirror), l^7 (half-row mirror), l^2, l^1.
constexpr int DPP_MIRROR = 0x140, DPP_HALF_MIRROR = 0x141, DPP_XOR2 = 0x4E, DPP_XOR1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ float row_sum16(float v) {
  v += dppf<DPP_MIRROR>(v);
  v += dppf<DPP_HALF_MIRROR>(v);
  v += dppf<DPP_XOR2>(v);
  v += dppf<DPP_XOR1>(v);
  return v;
}
__device__ __forceinline__ float row_max16(float v) {
  v = fmaxf(v, dppf<DPP_MIRROR>(v));
  v = fmaxf(v, dppf<DPP_HALF_MIRROR>(v));
  v = fmaxf(v, dppf<DPP_XOR2>(v));
  v = fmaxf(v, dppf<DPP_XOR1>(v));
  return v;
}
// (value, index) arg-max over the row: larger value, then lower index;
// index INT_MAX marks an empty entry.
template <int CTRL>
__device__ __forceinline__ void argmax_step(float& v, int& id) {
  const float v2 = dppf<CTRL>(v);
  const int i2 = dppi<CTRL>(id);
  const bool take = (i2 != 0x7fffffff) && (id == 0x7fffffff || v2 > v || (v2 == v && i2 < id));
  v = take ? v2 : v;
  id = take ? i2 : id;
}

// One stage of the reduce-scatter: the lane keeps half of its entries and
// adds the partner's copy of that half.
template <int W, int CTRL>
__device__ __forceinline__ void rs_stage(float (&pt)[16], bool up) {
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const float keep = up ? pt[W + i] : pt[i];
    const float send = up ? pt[i] : pt[W + i];
    pt[i] = keep + dppf<CTRL>(send);
  }
}

// Superposition of a prefix extended by one slot value v: MCA the max, MMCA
// the value of larger magnitude, the earlier on ties.  MCA's values are
// >= 0 (P is max(W, 0)), whose order is that of their bit patterns as
// signed integers: an integer max needs no NaN quieting of its operands.
template <bool MAG>
__device__ __forceinline__ float extend(float f, float v) {
  if constexpr (MAG) return (fabsf(v) > fabsf(f)) ? v : f;
  else return __int_as_float(max(__float_as_int(f), __float_as_int(v)));
}

// Depth-first enumeration of the K-subsets of the HP slots in lexicographic
// order; f is the superposition of the prefix MASK (DEPTH slots).
template <int HP, int NPIX, bool MAG, int K, int DEPTH, int LAST, unsigned MASK>
struct Enum {
  template <class V>
  static __device__ __forceinline__ void run(const float (&P)[HP][NPIX], const float (&f)[NPIX],
                                             V& v) {
    static_for<LAST + 1, HP - (K - DEPTH - 1)>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      float fc[NPIX];
#pragma unroll
      for (int i = 0; i < NPIX; ++i) {
        fc[i] = DEPTH == 0 ? P[j][i] : extend<MAG>(f[i], P[j][i]);
      }
      if constexpr (DEPTH + 1 == K) {
        v.template leaf<MASK | (1u << j)>(fc);
      } else {
        Enum<HP, NPIX, MAG, K, DEPTH + 1, j, MASK | (1u << j)>::run(P, fc, v);
      }
    });
  }
};

// Pass 1: residual of every state, reduce-scattered 16 states at a time;
// lane l keeps log-joint and residual of state 16 b + l in lj[b], rs[b].
template <int HP, int GAMMA, bool MAG, int NPIX>
struct Pass1 {
  static constexpr int NS = nstates_c(HP, GAMMA);
  static constexpr int NB = (NS + 15) / 16;
  const float (&y)[NPIX];
  int l;
  bool up8, up4, up2, up1;
  float c1, lam2;
  float mx;
  float pt[16];
  float lj[NB], rs[NB];

  __device__ __forceinline__ Pass1(const float (&y_)[NPIX], int l_, float c1_, float lam2_)
      : y(y_), l(l_), c1(c1_), lam2(lam2_), mx(-INFINITY) {
    up8 = (l & 8) != 0;
    up4 = (l & 4) != 0;
    up2 = (l & 2) != 0;
    up1 = (l & 1) != 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) pt[i] = 0.0f;
  }

  template <unsigned MASK>
  __device__ __forceinline__ void leaf(const float (&f)[NPIX]) {
    constexpr int c = canon_c(HP, MASK);
    float part = 0.0f;
#pragma unroll
    for (int i = 0; i < NPIX; ++i) {
      if constexpr (MAG) {
        part = __builtin_fmaf(f[i], __builtin_fmaf(-2.0f, y[i], f[i]), part);
      } else {
        const float r = y[i] - f[i];
        part = __builtin_fmaf(r, r, part);
      }
    }
    pt[c % 16] = part;
    if constexpr (c % 16 == 15 || c == NS - 1) flush<c / 16>();
  }

  template <int B>
  __device__ __forceinline__ void flush() {
    rs_stage<8, DPP_MIRROR>(pt, up8);
    rs_stage<4, DPP_HALF_MIRROR>(pt, up4);
    rs_stage<2, DPP_XOR2>(pt, up2);
    rs_stage<1, DPP_XOR1>(pt, up1);
    const int t = B * 16 + l;
    // number of actives of canonical state t
    int k = 0;
    static_for<1, GAMMA + 1>([&](auto kc) {
      constexpr int kk = decltype(kc)::value;
      k += t >= nstates_c(HP, kk - 1) ? 1 : 0;
    });
    const bool live = (B + 1) * 16 <= NS || t < NS;
    lj[B] = live ? (float)k * c1 - lam2 * pt[0] : -INFINITY;
    rs[B] = live ? pt[0] : 0.0f;
    mx = fmaxf(mx, lj[B]);
#pragma unroll
    for (int i = 0; i < 16; ++i) pt[i] = 0.0f;
  }
};

// Lane n of each row of 16 to the whole row (row_newbcast).
template <int N>
__device__ __forceinline__ float row_bcast(float v) {
  return dppf<0x150 + N>(v);
}

// Pass 2: responsibilities, walking the subset tree depth first (children
// of S add one slot above S's last).  The winner of a state at a pixel is
// the slot attaining the superposition there (the lower slot on ties; none
// while the superposition is 0).  A child S + j either takes over the win
// (its value beats S's superposition b) or inherits S's winner, and so do
// all of its descendants that do not take over later.  U(S) collects the
// weight of the states in S's subtree that inherit S's winner:
//   U(S) = sum over children c = S + j of [j does not beat b_S] (q(c) + U(c))
//   R[j] += [j beats b_S] (q(c) + U(c))
// and U(root) is dropped (no winner).
template <int HP, int NPIX, int NB>
struct Pass2 {
  float q[NB];  // lane l: posterior weight of state 16 b + l
  float thr;
  float R[HP][NPIX];
  template <int C>
  __device__ __forceinline__ float weight() const {
    return row_bcast<C % 16>(q[C / 16]);
  }
};

template <int HP, int GAMMA, int NPIX, bool MAG, int DEPTH, int LAST, unsigned MASK>
struct Resp {
  template <class V>
  static __device__ __forceinline__ void run(const float (&P)[HP][NPIX], const float (&b)[NPIX],
                                             float (&U)[NPIX], V& v) {
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr unsigned CM = MASK | (1u << j);
      const float qs = v.template weight<canon_c(HP, CM)>();
      if constexpr (DEPTH + 1 < GAMMA && j + 1 < HP) {
        float bc[NPIX], Uc[NPIX];
#pragma unroll
        for (int i = 0; i < NPIX; ++i) {
          bc[i] = DEPTH == 0 ? P[j][i] : extend<MAG>(b[i], P[j][i]);
          if constexpr (DEPTH > 0) asm volatile("" : "+v"(bc[i]));
          Uc[i] = qs;
        }
        Resp<HP, GAMMA, NPIX, MAG, DEPTH + 1, j, CM>::run(P, bc, Uc, v);
#pragma unroll
        for (int i = 0; i < NPIX; ++i) {
          const float pv = P[j][i];
          const bool cw = MAG ? (fabsf(pv) > fabsf(b[i])) : (pv > b[i]);
          v.R[j][i] += cw ? Uc[i] : 0.0f;
          U[i] += cw ? 0.0f : Uc[i];
          // pin each update at its place (else the backend sinks the whole
          // accumulation chains to their final use, keeping every term live)
          asm volatile("" : "+v"(v.R[j][i]), "+v"(U[i]));
        }
      } else {
        // no children: skipped where negligible at every point of the wave
        if (ballot64(qs > v.thr) != 0) {
#pragma unroll
          for (int i = 0; i < NPIX; ++i) {
            const float pv = P[j][i];
            const bool cw = MAG ? (fabsf(pv) > fabsf(b[i])) : (pv > b[i]);
            v.R[j][i] += cw ? qs : 0.0f;
            U[i] += cw ? 0.0f : qs;
            asm volatile("" : "+v"(v.R[j][i]), "+v"(U[i]));
          }
        }
      }
    });
  }
};

}  // namespace

// Adds the terms of this wave's points into the workgroup sums (plain LDS
// read-modify-write; the caller gives the wave exclusive access).  Points of
// the wave with the same latent in the same slot are added one at a time.
// One workgroup of 8 waves; with statistics, one workgroup per CU holding
// the LDS sums [A | B][HL][D] of latents < HL.
template <int HP, int GAMMA, bool MAG, int NPIX>
__global__ __launch_bounds__(512) void k_states_maxtree(
    const float* __restrict__ Y, int64_t N, int D, int Dp, const float* __restrict__ Pt32,
    const int32_t* __restrict__ sel, const uint32_t* __restrict__ tab_act,
    const Theta* __restrict__ th, float* __restrict__ s_mean, float* __restrict__ logL,
    uint32_t* __restrict__ top_mask, float* __restrict__ top_q, int topk, int accum, int HL,
    float* __restrict__ part, float* __restrict__ AT, float* __restrict__ BT, int Dq,
    double* __restrict__ scal) {
  constexpr int NS = nstates_c(HP, GAMMA);
  constexpr int NB = (NS + 15) / 16;
  extern __shared__ float acc_lds[];  // [A | B][HL][D]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l = lane & 15;
  const float c1 = th->c1_2, lam2 = th->lam2, beta = th->beta;
  const int nacc = 2 * HL * D;
  const bool lds_acc = accum && HL > 0;
  if (lds_acc) {
    for (int i = threadIdx.x; i < nacc; i += 512) acc_lds[i] = 0.0f;
    __syncthreads();
  }
  double acc_k = 0.0, acc_l = 0.0, acc_r = 0.0;

  for (int64_t sweep = (int64_t)blockIdx.x * 32; sweep < N; sweep += (int64_t)gridDim.x * 32) {
    const int64_t base = sweep + wave * 4;
    if (base >= N) break;  // past the end (later sweeps only go further)
    const int64_t n = base + g;
    const bool valid = n < N;
    const int64_t nn = valid ? n : N - 1;
    float y[NPIX];
    int hsel[HP];
    Pass2<HP, NPIX, NB> p2;
    {
      float P[HP][NPIX];
      {
#pragma unroll
        for (int j = 0; j < HP; ++j) hsel[j] = sel[nn * HP + j];
#pragma unroll
        for (int i = 0; i < NPIX; ++i) {
          const int d = l + 16 * i;
          y[i] = d < D ? Y[nn * D + d] : 0.0f;
        }
        // rows of P are zero beyond D and at least 16 NPIX long
#pragma unroll
        for (int j = 0; j < HP; ++j)
#pragma unroll
          for (int i = 0; i < NPIX; ++i) P[j][i] = Pt32[(int64_t)hsel[j] * Dp + l + 16 * i];
      }

      // ---- pass 1: log-joints (log2 units) and residuals of every state
      Pass1<HP, GAMMA, MAG, NPIX> p1(y, l, c1, lam2);
      {
        float zero[NPIX];
#pragma unroll
        for (int i = 0; i < NPIX; ++i) zero[i] = 0.0f;
        p1.template leaf<0u>(zero);
        static_for<1, GAMMA + 1>([&](auto kc) {
          constexpr int K = decltype(kc)::value;
          // fresh identities for P per cardinality (no instruction): value
          // numbering would otherwise share the prefixes of one cardinality
          // with the next and keep them all live in between
#pragma unroll
          for (int j = 0; j < HP; ++j)
#pragma unroll
            for (int i = 0; i < NPIX; ++i) asm volatile("" : "+v"(P[j][i]));
          Enum<HP, NPIX, MAG, K, 0, -1, 0u>::run(P, zero, p1);
        });
      }
      const float m = row_max16(p1.mx);
      float z = 0.0f, z1 = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float dd = p1.lj[b] - m;  // -inf for the padding entries
        z1 += __builtin_amdgcn_exp2f(dd);
        z += beta == 1.0f ? __builtin_amdgcn_exp2f(dd) : __builtin_amdgcn_exp2f(beta * dd);
      }
      const float Z = row_sum16(z);
      const float Z1 = beta == 1.0f ? Z : row_sum16(z1);
      const float invZ = 1.0f / Z;

      // ---- top-k: repeated arg-max below the previous winner in (lj desc, index asc)
      if (topk > 0) {
        float pv = INFINITY;
        int pid = -1;
        for (int t = 0; t < topk; ++t) {
          float v = -INFINITY;
          int id = 0x7fffffff;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int k = 16 * b + l;
            const float x = p1.lj[b];
            const bool below = (x < pv) || (x == pv && k > pid);
            if (k < NS && below && (x > v || id == 0x7fffffff)) {
              v = x;
              id = k;
            }
          }
          argmax_step<DPP_MIRROR>(v, id);
          argmax_step<DPP_HALF_MIRROR>(v, id);
          argmax_step<DPP_XOR2>(v, id);
          argmax_step<DPP_XOR1>(v, id);
          if (l == 0 && valid) {
            if (top_q) top_q[n * topk + t] = __builtin_amdgcn_exp2f(beta * (v - m)) * invZ;
            if (top_mask) top_mask[n * topk + t] = tab_act[id];
          }
          pv = v;
          pid = id;
        }
      }

      // ---- q, moments, expected residual
      float res = 0.0f;
      float sm[HP];
#pragma unroll
      for (int j = 0; j < HP; ++j) sm[j] = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = 16 * b + l;
        const float qv = __builtin_amdgcn_exp2f(beta * (p1.lj[b] - m)) * invZ;  // 0 on padding
        res = __builtin_fmaf(qv, p1.rs[b], res);
        const uint32_t act = t < NS ? tab_act[t] : 0u;
#pragma unroll
        for (int j = 0; j < HP; ++j) sm[j] += ((act >> j) & 1u) ? qv : 0.0f;
        p2.q[b] = qv;
      }
      float kmean = 0.0f;
#pragma unroll
      for (int j = 0; j < HP; ++j) {
        sm[j] = row_sum16(sm[j]);
        kmean += sm[j];
      }
      if (valid) {
#pragma unroll
        for (int j = 0; j < HP; ++j)
          if (l == j) s_mean[n * HP + j] = sm[j];
      }
      const float resid = row_sum16(res);  // <||y - f(s)||^2>, relative to ||y||^2 for MMCA
      double yy_n = 0.0;  // ||y||^2 in FP64 (MMCA: added back to logL and the residual)
      if constexpr (MAG) {
#pragma unroll
        for (int i = 0; i < NPIX; ++i) yy_n += (double)y[i] * (double)y[i];
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) yy_n += __shfl_xor(yy_n, o, 64);
      }
      const double lL = th->c0 + 0.6931471805599453 * ((double)m + (double)log2f(Z1) -
                                                       (double)lam2 * yy_n);
      if (l == 0 && valid) {
        if (logL) logL[n] = (float)lL;
        acc_k += kmean;
        acc_l += lL;
        acc_r += (double)resid + yy_n;
      }

      // ---- pass 2: responsibilities
      if (accum) {
        // P read again (from L2): nothing of pass 1 stays live across the
        // log-sum-exp, and value numbering cannot carry pass 1's maxima over
        // to the equal ones here
#pragma unroll
        for (int j = 0; j < HP; ++j) {
          hsel[j] = sel[nn * HP + j];
#pragma unroll
          for (int i = 0; i < NPIX; ++i) P[j][i] = Pt32[(int64_t)hsel[j] * Dp + l + 16 * i];
        }
        // 2^-40 of the largest weight of this point (1/Z: the best state's)
        p2.thr = valid ? 0x1p-40f * invZ : INFINITY;
#pragma unroll
        for (int j = 0; j < HP; ++j)
#pragma unroll
          for (int i = 0; i < NPIX; ++i) p2.R[j][i] = 0.0f;
        float b0[NPIX], U0[NPIX];
#pragma unroll
        for (int i = 0; i < NPIX; ++i) {
          b0[i] = 0.0f;
          U0[i] = 0.0f;
        }
        Resp<HP, GAMMA, NPIX, MAG, 0, -1, 0u>::run(P, b0, U0, p2);
        if (valid) {
#pragma unroll
          for (int j = 0; j < HP; ++j) {
            const int h = hsel[j];
            if (h < HL) {
              float* la = acc_lds + h * D;
              float* lb = acc_lds + (HL + h) * D;
#pragma unroll
              for (int i = 0; i < NPIX; ++i) {
                const int d = l + 16 * i;
                const float r = p2.R[j][i];
                if (d < D && r != 0.0f) {
                  atomicAdd(la + d, r * y[i]);
                  atomicAdd(lb + d, r);
                }
              }
            } else {
              float* at = AT + (int64_t)(h - HL) * Dq;
              float* bt = BT + (int64_t)(h - HL) * Dq;
#pragma unroll
              for (int i = 0; i < NPIX; ++i) {
                const int d = l + 16 * i;
                const float r = p2.R[j][i];
                if (d < D && r != 0.0f) {
                  atomicAdd(at + d, r * y[i]);
                  atomicAdd(bt + d, r);
                }
              }
            }
          }
        }
      }
    }
  }
  if (scal && l == 0) {
    atomicAdd(&scal[0], acc_k);
    atomicAdd(&scal[1], acc_l);
    atomicAdd(&scal[3], acc_r);
  }
  if (lds_acc) {
    __syncthreads();
    float* dst = part + (int64_t)blockIdx.x * nacc;
    for (int i = threadIdx.x; i < nacc; i += 512) dst[i] = acc_lds[i];
  }
}

// A[d][h] += sum over workgroups of their sums (latents < HL), added in FP64.
// Each block takes 64 entries; its four waves sum a quarter of the
// workgroup sums each.
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int nparts,
                                                      int HL, int D, int H,
                                                      float* __restrict__ A,
                                                      float* __restrict__ B) {
  __shared__ double red[4][64];
  const int nacc = 2 * HL * D;
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;
  double s0 = 0.0, s1 = 0.0;
  if (e < nacc) {
    int w = q;
    for (; w + 4 < nparts; w += 8) {
      s0 += (double)part[(int64_t)w * nacc + e];
      s1 += (double)part[(int64_t)(w + 4) * nacc + e];
    }
    if (w < nparts) s0 += (double)part[(int64_t)w * nacc + e];
  }
  red[q][threadIdx.x & 63] = s0 + s1;
  __syncthreads();
  if (q == 0 && e < nacc) {
    const double tot = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                       red[3][threadIdx.x];
    const int which = e / (HL * D);
    const int r = e - which * HL * D;
    const int h = r / D, d = r - h * D;
    float* dst = which ? B : A;
    dst[(int64_t)d * H + h] += (float)tot;
  }
}

// Fill of the transposed accumulators (a kernel, so that the call can be
// captured in a graph).
__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.0f;
}

// A[d][HL + h] += AT[h][d], B[d][HL + h] += BT[h][d] for h < H - HL.
__global__ __launch_bounds__(256) void k_add_transposed(const float* __restrict__ AT,
                                                        const float* __restrict__ BT, int Dq,
                                                        int D, int H, int HL,
                                                        float* __restrict__ A,
                                                        float* __restrict__ B) {
  __shared__ float ta[32][33], tb[32][33];
  const int HR = H - HL;
  const int h0 = blockIdx.x * 32, d0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int h = h0 + r, d = d0 + tx;
    const bool ok = h < HR && d < D;
    ta[r][tx] = ok ? AT[(int64_t)h * Dq + d] : 0.0f;
    tb[r][tx] = ok ? BT[(int64_t)h * Dq + d] : 0.0f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, h = h0 + tx;
    if (d < D && h < HR) {
      A[(int64_t)d * H + HL + h] += ta[tx][r];
      B[(int64_t)d * H + HL + h] += tb[tx][r];
    }
  }
}

// Shapes with a compiled walk: (H', gamma) and the pixels per lane.
#define PROSPER_MAXTREE_SHAPES(X) X(10, 3)

static int maxtree_npix(int D) {
  if (D <= 64) return 4;
  if (D <= 112) return 7;
  if (D <= 128) return 8;
  return 0;
}

bool has_max_tree(int Hp, int gamma, int D, int H) {
  if (maxtree_npix(D) == 0) return false;
  if (Hp == H && gamma == Hp) return false;  // the all-active state takes the table walk
#define X(HPV, GV) \
  if (Hp == HPV && gamma == GV) return true;
  PROSPER_MAXTREE_SHAPES(X)
#undef X
  return false;
}

// LDS of the statistics workgroups: 160 KB, of which the sums take what fits.
static constexpr int MAXTREE_LDS_FLOATS = 160 * 1024 / 4;
static int maxtree_hl(int D, int H) {
  const int hl = MAXTREE_LDS_FLOATS / (2 * D);
  return hl < H ? hl : H;
}

// Scratch of the statistics (in floats): the workgroup sums, then the
// transposed sums of the latents beyond LDS.
size_t max_tree_acc_floats(int D, int H, int nparts) {
  const int HL = maxtree_hl(D, H);
  return (size_t)nparts * 2 * HL * D + 2 * (size_t)(H - HL) * round_up(D, 16);
}

template <int HP, int GAMMA, bool MAG, int NPIX>
static hipError_t launch_mt(const float* Y, int64_t N, int D, int Dp, const Prepared& p,
                            const Scratch& s, const uint32_t* tab_act, float* logL,
                            uint32_t* top_mask, float* top_q, int topk, int accum, int HL,
                            int blocks, float* part, float* AT, float* BT, int Dq,
                            double* scal, hipStream_t st) {
  auto kern = k_states_maxtree<HP, GAMMA, MAG, NPIX>;
  const size_t lds = accum ? (size_t)2 * HL * D * 4 : 0;
  hipError_t e0 = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(512), lds, st, Y, N, D, Dp, p.Pt32,
                     s.sel, tab_act, p.theta, s.s_mean, logL, top_mask, top_q, topk, accum, HL,
                     part, AT, BT, Dq, scal);
  return hipGetLastError();
}

hipError_t launch_states_max_tree(int model, int Hp, int gamma, int64_t N, int D, int Dp, int H,
                                  const uint32_t* tab_act, const float* Y, const Prepared& p,
                                  const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                                  int topk, float* A_num, float* B_den, double* scal,
                                  hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int npix = maxtree_npix(D);
  const bool mag = model == PROSPER_MMCA;
  const int Dq = round_up(D, 16);
  const int64_t groups = (N + 31) / 32;  // 32 points per workgroup and sweep
  const int accum = A_num != nullptr ? 1 : 0;
  int HL = 0, blocks;
  float *part = nullptr, *AT = nullptr, *BT = nullptr;
  if (accum) {
    if (!s.max_acc || s.max_parts <= 0) return hipErrorInvalidValue;
    HL = maxtree_hl(D, H);
    blocks = (int)(groups < s.max_parts ? groups : s.max_parts);
    part = s.max_acc;
    AT = part + (size_t)s.max_parts * 2 * HL * D;
    BT = AT + (size_t)(H - HL) * Dq;
    if (H > HL) {
      const int64_t nf = 2 * (int64_t)(H - HL) * Dq;
      const int64_t fb = (nf + 255) / 256;
      hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(fb < 1024 ? fb : 1024)), dim3(256), 0,
                         st, AT, nf);
    }
  } else {
    blocks = (int)(groups < 2048 ? groups : 2048);
  }
  hipError_t e = hipErrorInvalidValue;
#define LAUNCH(HPV, GV, NP)                                                                    \
  (mag ? launch_mt<HPV, GV, true, NP>(Y, N, D, Dp, p, s, tab_act, logL, top_mask, top_q, topk, \
                                      accum, HL, blocks, part, AT, BT, Dq, scal, st)           \
       : launch_mt<HPV, GV, false, NP>(Y, N, D, Dp, p, s, tab_act, logL, top_mask, top_q,      \
                                       topk, accum, HL, blocks, part, AT, BT, Dq, scal, st))
#define X(HPV, GV)                       \
  if (Hp == HPV && gamma == GV) {        \
    if (npix == 4)                       \
      e = LAUNCH(HPV, GV, 4);            \
    else if (npix == 7)                  \
      e = LAUNCH(HPV, GV, 7);            \
    else if (npix == 8)                  \
      e = LAUNCH(HPV, GV, 8);            \
  }
  PROSPER_MAXTREE_SHAPES(X)
#undef X
#undef LAUNCH
  if (e != hipSuccess || !accum) return e;
  if (HL > 0) {
    const int nacc = 2 * HL * D;
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((nacc + 63) / 64)), dim3(256), 0, st,
                       part, blocks, HL, D, H, A_num, B_den);
  }
  if (H > HL) {
    dim3 grid((unsigned)((H - HL + 31) / 32), (unsigned)((D + 31) / 32));
    hipLaunchKernelGGL(k_add_transposed, grid, dim3(256), 0, st, AT, BT, Dq, D, H, HL, A_num,
                       B_den);
  }
  return hipGetLastError();
}

}  // namespace prosper
