// State walk for max superposition (MCA): rows a4-a8 of the hot path.
//
// f_d(s) = max_h s_h W_dh.  For a state with k < H active latents the
// inactive ones contribute 0 to the max, so f_d = max(0, max_{j in s} P_dj)
// with P = max(W, 0), the rows the projection ranked.  The state with all H
// latents active (reachable only when H' = H = gamma) has no inactive latent:
// its superposition is max_h W_dh of the unclamped W, which is negative on a
// pixel whose whole row of W is negative; the parameter preparation stores
// that row maximum (wmax) and the walk takes it for this state.  The log-joint is taken
// with the direct residual (log2 units, up to the constant c0):
//   lj(s) = k(s) c1 - lam ||y - f(s)||^2                   (Eq. 1 + Eq. 2)
// Unlike the linear models, the form relative to the zero state would carry
// lam ||y||^2 (hundreds to thousands) in every FP32 log-joint, whose rounding
// alone would exceed the FP32 tolerance; the direct residual is small for
// every state that carries posterior mass.
// No contraction structure exists here (a max, not a sum, over the active
// components), so this is a VALU kernel without MFMA: one wave per data
// point, lanes over pixels, the H' candidate columns of P staged in LDS.
// States are processed 64 at a time: every lane forms its pixel-partial sum
// for each of the 64 states and a butterfly reduce-scatter leaves the full
// sum of state t in lane t.
//
// Responsibilities for the M-step (hard-max limit of the smooth maximum):
//   R[d][j] = sum_s q(s) [slot j is the lowest-index active slot attaining
//             max_{j in s} P_dj, and that max is > 0]
// accumulated as A_num[d][c_j] += R y_d and B_den[d][c_j] += R, plus
// sum_s q(s) ||y - f(s)||^2 for the noise update.
//
// MMCA (MAG = true): f_d(s) is the s_h W_dh of largest magnitude, the lower
// slot on equal magnitudes, and 0 for the zero state; P is W itself (no clamp).
// The responsibility of pixel d goes to the active slot of largest |P_dj|
// when that magnitude is > 0; statistics and M-step are those of MCA.
// With both signs in W every pixel of an active state differs from y, so the
// walk sums the residual relative to the zero state, sum_d mu_d (mu_d - 2 y_d),
// which stays small where ||y||^2 would dominate FP32 rounding; lam ||y||^2
// (reduced in FP64) is added back to logL and to the expected residual.
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

static constexpr int MCA_ND = 16;  // pixels per lane (D <= 1024)

template <bool MAG>
__global__ __launch_bounds__(64) void k_states_max(
    const float* __restrict__ Y, int64_t N, int D, int Dp, int H, int Hp, int64_t nstates,
    const uint32_t* __restrict__ tab_act, const float* __restrict__ Pt32,
    const float* __restrict__ wmax, const int32_t* __restrict__ sel, const float* __restrict__ yy, const Theta* __restrict__ th,
    float* __restrict__ s_mean, float* __restrict__ logL, uint32_t* __restrict__ top_mask,
    float* __restrict__ top_q, int topk, float* __restrict__ A_num, float* __restrict__ B_den,
    double* __restrict__ scal) {
  extern __shared__ float sm[];
  float* Pc = sm;                                 // [Hp][D]
  const int64_t ns4 = (nstates + 3) & ~(int64_t)3;
  float* ljs = Pc + Hp * D;                       // [nstates]: lj, then q
  float* Rs = ljs + ns4;                          // [nstates]: ||y - f(s)||^2
  float* Rl = Rs + ns4;                           // [Hp][D] (accumulation only)
  const int lane = threadIdx.x;
  const float lam2 = th->lam2, c1 = th->c1_2;
  const int nd = (D + 63) / 64;
  double acc_k = 0.0, acc_l = 0.0, acc_r = 0.0;

  for (int64_t n = blockIdx.x; n < N; n += gridDim.x) {
    float yv[MCA_ND];
#pragma unroll
    for (int i = 0; i < MCA_ND; ++i) {
      const int d = lane + 64 * i;
      yv[i] = (i < nd && d < D) ? Y[n * D + d] : 0.0f;
    }
    for (int j = 0; j < Hp; ++j) {
      const int h = sel[n * Hp + j];
      for (int d = lane; d < D; d += 64) {
        Pc[j * D + d] = Pt32[(int64_t)h * Dp + d];
        if (A_num) Rl[j * D + d] = 0.0f;
      }
    }
    __syncthreads();
    // ---- log-joints, 64 states per round
    float mx = -INFINITY;
    for (int64_t k0 = 0; k0 < nstates; k0 += 64) {
      float pt[64];
#pragma unroll
      for (int t = 0; t < 64; ++t) {
        const int64_t k = k0 + t;
        float part = 0.0f;
        if (k < nstates) {
          const uint32_t act = tab_act[k];
          const bool floor0 = __popc(act) < H;
#pragma unroll
          for (int i = 0; i < MCA_ND; ++i) {
            const int d = lane + 64 * i;
            if (i < nd && d < D) {
              float mu = 0.0f;
              uint32_t rem = act;
              if (!MAG && !floor0) {
                mu = wmax[d];
                rem = 0u;
              }
              while (rem) {
                const int j = __ffs(rem) - 1;
                rem &= rem - 1u;
                const float v = Pc[j * D + d];
                if (MAG)
                  mu = (fabsf(v) > fabsf(mu)) ? v : mu;
                else
                  mu = fmaxf(mu, v);
              }
              if (MAG) {
                part = __builtin_fmaf(mu, mu - 2.0f * yv[i], part);
              } else {
                const float r = yv[i] - mu;
                part = __builtin_fmaf(r, r, part);
              }
            }
          }
        }
        pt[t] = part;
      }
      // butterfly reduce-scatter: lane t ends with the pixel sum of state k0 + t
#pragma unroll
      for (int w = 32; w >= 1; w >>= 1) {
        const bool up = (lane & w) != 0;
#pragma unroll
        for (int i = 0; i < w; ++i) {
          const float keep = up ? pt[w + i] : pt[i];
          const float send = up ? pt[i] : pt[w + i];
          pt[i] = keep + __shfl_xor(send, w, 64);
        }
      }
      const int64_t k = k0 + lane;
      if (k < nstates) {
        const float lj = (float)__popc(tab_act[k]) * c1 - lam2 * pt[0];
        ljs[k] = lj;
        Rs[k] = pt[0];
        mx = fmaxf(mx, lj);
      }
    }
    __syncthreads();
    const float m = wave_max(mx);
    // annealing: q from 2^(beta (lj - m)), logL from the untempered sum
    const float beta = th->beta;
    float z = 0.0f, z1 = 0.0f;
    for (int64_t k = lane; k < nstates; k += 64) {
      const float d = ljs[k] - m;
      z1 += __builtin_amdgcn_exp2f(d);
      z += beta == 1.0f ? __builtin_amdgcn_exp2f(d) : __builtin_amdgcn_exp2f(beta * d);
    }
    const float Z = wave_sum(z);
    const float Z1 = beta == 1.0f ? Z : wave_sum(z1);
    const float invZ = 1.0f / Z;
    // ---- top-k: repeated arg-max below the previous winner in (lj desc, index asc)
    {
      float pv = INFINITY;
      int pid = -1;
      for (int t = 0; t < topk; ++t) {
        float v = -INFINITY;
        int id = 0x7fffffff;
        for (int64_t k = lane; k < nstates; k += 64) {
          const float x = ljs[k];
          const bool below = (x < pv) || (x == pv && (int)k > pid);
          if (below && (x > v || id == 0x7fffffff)) {
            v = x;
            id = (int)k;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const float v2 = __shfl_xor(v, o, 64);
          const int i2 = __shfl_xor(id, o, 64);
          const bool take = (i2 != 0x7fffffff) &&
                            (id == 0x7fffffff || v2 > v || (v2 == v && i2 < id));
          v = take ? v2 : v;
          id = take ? i2 : id;
        }
        if (lane == 0) {
          if (top_q) top_q[n * topk + t] = __builtin_amdgcn_exp2f(beta * (v - m)) * invZ;
          if (top_mask) top_mask[n * topk + t] = tab_act[id];
        }
        pv = v;
        pid = id;
      }
    }
    __syncthreads();
    // ---- q, moments, expected residual
    float res = 0.0f;
    for (int64_t k = lane; k < nstates; k += 64) {
      const float q = __builtin_amdgcn_exp2f(beta * (ljs[k] - m)) * invZ;
      res += q * Rs[k];
      ljs[k] = q;
    }
    __syncthreads();
    float kmean = 0.0f;
    for (int j = 0; j < Hp; ++j) {
      float part = 0.0f;
      for (int64_t k = lane; k < nstates; k += 64)
        if ((tab_act[k] >> j) & 1u) part += ljs[k];
      part = wave_sum(part);
      kmean += part;
      if (lane == 0) s_mean[n * Hp + j] = part;
    }
    const float resid = wave_sum(res);  // <||y - f(s)||^2>, relative to ||y||^2 if MAG
    double yy_n = 0.0;
    if (MAG) {
#pragma unroll
      for (int i = 0; i < MCA_ND; ++i) yy_n += (double)yv[i] * (double)yv[i];
      for (int w = 32; w >= 1; w >>= 1) yy_n += __shfl_xor(yy_n, w, 64);
    }
    const double lL = th->c0 + 0.6931471805599453 * ((double)m + (double)log2f(Z1) -
                                                     (double)lam2 * yy_n);
    if (lane == 0) {
      if (logL) logL[n] = (float)lL;
      acc_k += kmean;
      acc_l += lL;
      acc_r += (double)resid + yy_n;
    }
    // ---- responsibilities
    if (A_num) {
      for (int64_t k = 0; k < nstates; ++k) {
        const uint32_t act = tab_act[k];
        if (!act) continue;
        const float q = ljs[k];
#pragma unroll
        for (int i = 0; i < MCA_ND; ++i) {
          const int d = lane + 64 * i;
          if (i < nd && d < D) {
            float best = MAG ? 0.0f : -INFINITY;
            int bj = -1;
            uint32_t rem = act;
            while (rem) {
              const int j = __ffs(rem) - 1;
              rem &= rem - 1u;
              const float v = MAG ? fabsf(Pc[j * D + d]) : Pc[j * D + d];
              if (v > best) {
                best = v;
                bj = j;
              }
            }
            if (best > 0.0f) Rl[bj * D + d] += q;
          }
        }
      }
      for (int j = 0; j < Hp; ++j) {
        const int h = sel[n * Hp + j];
#pragma unroll
        for (int i = 0; i < MCA_ND; ++i) {
          const int d = lane + 64 * i;
          if (i < nd && d < D) {
            const float r = Rl[j * D + d];
            if (r != 0.0f) {
              atomicAdd(&A_num[(int64_t)d * H + h], r * yv[i]);
              atomicAdd(&B_den[(int64_t)d * H + h], r);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (scal && lane == 0) {
    atomicAdd(&scal[0], acc_k);
    atomicAdd(&scal[1], acc_l);
    atomicAdd(&scal[3], acc_r);
  }
}

size_t states_max_lds_bytes(int Hp, int D, int64_t nstates, bool acc) {
  return ((size_t)Hp * D + 2 * (size_t)((nstates + 3) & ~(int64_t)3) + (acc ? (size_t)Hp * D : 0)) * 4;
}

hipError_t launch_states_max(int model, int Hp, int gamma, int64_t N, int D, int Dp, int H, int64_t nstates,
                             const uint32_t* tab_act, const float* Y, const Prepared& p,
                             const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, float* A_num, float* B_den, double* scal,
                             hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (has_max_tree(Hp, gamma, D, H) && (A_num == nullptr || s.max_acc != nullptr))
    return launch_states_max_tree(model, Hp, gamma, N, D, Dp, H, tab_act, Y, p, s, logL,
                                  top_mask, top_q, topk, A_num, B_den, scal, st);
  const size_t lds = states_max_lds_bytes(Hp, D, nstates, A_num != nullptr);
  const bool mag = model == PROSPER_MMCA;
  const auto kern = mag ? k_states_max<true> : k_states_max<false>;
  hipError_t e0 = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
  if (e0 != hipSuccess) return e0;
  int64_t blocks = N < 8192 ? N : 8192;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64), lds, st, Y, N, D, Dp, H, Hp,
                     nstates, tab_act, p.Pt32, p.wmax, s.sel, s.yy, p.theta, s.s_mean, logL, top_mask,
                     top_q, topk, A_num, B_den, scal);
  return hipGetLastError();
}

}  // namespace prosper
