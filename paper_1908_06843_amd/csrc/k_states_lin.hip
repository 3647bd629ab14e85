// State walk for linear superposition (BSC, TSC): rows a4-a8 of the hot path.
//
// For each point the log-joint of every state of the truncated set K_n is
// needed (Eq. 1 + Eq. 2 with f = W s).  Relative to the zero state and in
// log2 units it decomposes into singleton and pair terms of the H'
// candidates (j, j' are slots, c_j = I_n(j), b = W^T y, G = W^T W):
//   lj(s) = sum_j [c1 + lam (2 s_j b_cj - G_cjcj)] + sum_{j<j'} s_j s_j' (-2 lam G_cjcj')
// so only b on the candidates and the H' x H' block of G enter.  The
// posterior q = 2^(lj - m) / Z (m = max lj, Z = sum 2^(lj - m)) gives
//   <s_j> = sum_s q s_j,  <s_j s_j'> = sum_s q s_j s_j',  logL = lj(0) + ln2 (m + log2 Z).
//
// Two implementations:
//  * k_states_tree<H', gamma, ...> (k_states_tree.hpp, one translation unit
//    per shape): one lane per data point, the state set unrolled at compile
//    time as a depth-first walk of the subset tree, every operand a register.
//  * k_states_generic: one wave per data point, lanes over the canonical
//    state table, singleton/pair terms in LDS.  Any H' <= 32 and |K|.
#include "k_states_tree.hpp"

namespace prosper {

// ----------------------------------------------------------------- generic
// One wave per point; lanes stride over the canonical table.  LDS per wave:
// singleton terms (u+ / u-), pair terms and the moment accumulators.
struct GenLds {
  float up[32], um[32];
  float p[32 * 32];
  float M[32], K2[32];
  float P[32 * 32];
};

template <bool TSC>
__global__ __launch_bounds__(256) void k_states_generic(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, int Hp, int64_t nstates,
    const uint32_t* __restrict__ tab_act, const uint32_t* __restrict__ tab_sgn,
    const Theta* __restrict__ th, float* __restrict__ s_mean, float* __restrict__ logL,
    uint32_t* __restrict__ top_mask, float* __restrict__ top_q, int topk,
    float* __restrict__ ss_out, float* __restrict__ B_atomic, double* __restrict__ scal,
    const int32_t* __restrict__ list, const int32_t* __restrict__ list_count,
    float* __restrict__ k_out, float* __restrict__ res_out) {
  __shared__ GenLds sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  GenLds& S = sh[wave];
  const float lam2 = th->lam2, c1 = th->c1_2;
  // annealing: moments under 2^(beta (lj - m)), logL from the untempered sum
  const float beta = th->beta;
  const bool tempered = beta != 1.0f;
  const int64_t Ntot = N;  // leading dimension of ss_out
  double acc_k = 0.0, acc_l = 0.0;
  // list mode: only the points named in list[0 .. *list_count)
  const int64_t npts = list ? (int64_t)*list_count : N;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < npts; base += (int64_t)gridDim.x * 4) {
    const bool live = base + wave < npts;
    const int64_t n = !live ? 0 : (list ? (int64_t)list[base + wave] : base + wave);
    if (live) {
      for (int j = lane; j < Hp; j += 64) {
        const int sj = sel[n * Hp + j];
        const float g = G[(int64_t)sj * H + sj];
        const float bj = bc[n * Hp + j];
        S.up[j] = c1 + lam2 * (2.0f * bj - g);
        S.um[j] = c1 + lam2 * (-2.0f * bj - g);
        S.M[j] = 0.0f;
        S.K2[j] = 0.0f;
      }
      for (int idx = lane; idx < Hp * Hp; idx += 64) {
        const int i = idx / Hp, j = idx % Hp;
        if (i < j) {
          S.p[i * 32 + j] = -2.0f * lam2 * G[(int64_t)sel[n * Hp + i] * H + sel[n * Hp + j]];
          S.P[i * 32 + j] = 0.0f;
        }
      }
    }
    __syncthreads();
    // pass 1: max and per-lane top list
    float mx = -INFINITY;
    float tv[PROSPER_MAX_TOPK];
    int ti[PROSPER_MAX_TOPK];
#pragma unroll
    for (int t = 0; t < PROSPER_MAX_TOPK; ++t) {
      tv[t] = -INFINITY;
      ti[t] = 0x7fffffff;
    }
    if (live) {
      for (int64_t k = lane; k < nstates; k += 64) {
        const uint32_t act = tab_act[k];
        const uint32_t sg = TSC ? tab_sgn[k] : 0u;
        float L = 0.0f;
        uint32_t rem = act;
        while (rem) {
          const int j = __ffs(rem) - 1;
          rem &= rem - 1u;
          const bool nj = (sg >> j) & 1u;
          L += nj ? S.um[j] : S.up[j];
          uint32_t pre = act & ((1u << j) - 1u);
          while (pre) {
            const int i = __ffs(pre) - 1;
            pre &= pre - 1u;
            const bool ni = (sg >> i) & 1u;
            const float v = S.p[i * 32 + j];
            L += (ni != nj) ? -v : v;
          }
        }
        mx = fmaxf(mx, L);
        if (topk > 0) {
          float v = L;
          int id = (int)k;
#pragma unroll
          for (int t = 0; t < PROSPER_MAX_TOPK; ++t) {
            const bool better = v > tv[t];  // lane visits states in increasing index
            const float v2 = better ? tv[t] : v;
            const int i2 = better ? ti[t] : id;
            tv[t] = better ? v : tv[t];
            ti[t] = better ? id : ti[t];
            v = v2;
            id = i2;
          }
        }
      }
    }
    const float m = wave_max(mx);
    // pass 2: weights and moments (zl: the weighted log-joints, for res_out)
    float z = 0.0f, z1 = 0.0f, zl = 0.0f;
    if (live) {
      for (int64_t k = lane; k < nstates; k += 64) {
        const uint32_t act = tab_act[k];
        const uint32_t sg = TSC ? tab_sgn[k] : 0u;
        float L = 0.0f;
        uint32_t rem = act;
        while (rem) {
          const int j = __ffs(rem) - 1;
          rem &= rem - 1u;
          const bool nj = (sg >> j) & 1u;
          L += nj ? S.um[j] : S.up[j];
          uint32_t pre = act & ((1u << j) - 1u);
          while (pre) {
            const int i = __ffs(pre) - 1;
            pre &= pre - 1u;
            const bool ni = (sg >> i) & 1u;
            const float v = S.p[i * 32 + j];
            L += (ni != nj) ? -v : v;
          }
        }
        const float e1 = fast_exp2(L - m);
        const float e = tempered ? fast_exp2(beta * (L - m)) : e1;
        z += e;
        z1 += e1;
        zl = fmaf(e, L, zl);
        rem = act;
        while (rem) {
          const int j = __ffs(rem) - 1;
          rem &= rem - 1u;
          const bool nj = (sg >> j) & 1u;
          atomicAdd(&S.M[j], nj ? -e : e);
          if (TSC) atomicAdd(&S.K2[j], e);
          uint32_t pre = act & ((1u << j) - 1u);
          while (pre) {
            const int i = __ffs(pre) - 1;
            pre &= pre - 1u;
            const bool ni = (sg >> i) & 1u;
            atomicAdd(&S.P[i * 32 + j], (ni != nj) ? -e : e);
          }
        }
      }
    }
    const float Z = wave_sum(z);
    const float Z1 = tempered ? wave_sum(z1) : Z;
    __syncthreads();
    if (live) {
      const float invZ = 1.0f / Z;
      const double lL = th->c0 - (double)th->lam * (double)yy[n] +
                        0.6931471805599453 * ((double)m + (double)log2f(Z1));
      float kpart = 0.0f;
      for (int j = lane; j < Hp; j += 64) {
        const float k2 = TSC ? S.K2[j] : S.M[j];
        kpart += k2;
        s_mean[n * Hp + j] = S.M[j] * invZ;
        if (ss_out) ss_out[(int64_t)j * Ntot + n] = k2 * invZ;
        if (B_atomic) {
          const int sj = sel[n * Hp + j];
          atomicAdd(&B_atomic[(int64_t)sj * H + sj], k2 * invZ);
        }
      }
      if (B_atomic) {  // few points (the exact kernel's redo list): direct adds
        for (int idx = lane; idx < Hp * Hp; idx += 64) {
          const int i = idx / Hp, j = idx % Hp;
          if (i < j)
            atomicAdd(&B_atomic[(int64_t)sel[n * Hp + i] * H + sel[n * Hp + j]],
                      S.P[i * 32 + j] * invZ);
        }
      }
      if (ss_out) {  // pairs i < j in row-major order after the diagonal
        for (int idx = lane; idx < Hp * Hp; idx += 64) {
          const int i = idx / Hp, j = idx % Hp;
          if (i < j) {
            const int p = Hp + i * (2 * Hp - i - 1) / 2 + (j - i - 1);
            ss_out[(int64_t)p * Ntot + n] = S.P[i * 32 + j] * invZ;
          }
        }
      }
      const float kmean = wave_sum(kpart) * invZ;
      // <||y - W s||^2> = ||y||^2 - <2 s^T b - s^T G s>, and the log-joint
      // relative to the zero state is k c1 + lam2 (2 s^T b - s^T G s)
      const float EL = res_out ? wave_sum(zl) * invZ : 0.0f;
      if (lane == 0) {
        if (logL) logL[n] = (float)lL;
        if (k_out) k_out[n] = kmean;
        if (res_out)
          res_out[n] = (float)((double)yy[n] - ((double)EL - (double)c1 * (double)kmean) /
                                                   (double)lam2);
        acc_k += kmean;
        acc_l += lL;
      }
      // top-k merge: repeated wave arg-max over the lanes' list heads
      for (int t = 0; t < topk; ++t) {
        float v = tv[0];
        int id = ti[0];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const float v2 = __shfl_xor(v, o, 64);
          const int i2 = __shfl_xor(id, o, 64);
          const bool take = (v2 > v) || (v2 == v && i2 < id);
          v = take ? v2 : v;
          id = take ? i2 : id;
        }
        if (ti[0] == id) {  // the winner pops its head
#pragma unroll
          for (int s2 = 0; s2 + 1 < PROSPER_MAX_TOPK; ++s2) {
            tv[s2] = tv[s2 + 1];
            ti[s2] = ti[s2 + 1];
          }
          tv[PROSPER_MAX_TOPK - 1] = -INFINITY;
          ti[PROSPER_MAX_TOPK - 1] = 0x7fffffff;
        }
        if (lane == 0) {
          if (top_q) top_q[n * topk + t] = fast_exp2((tempered ? beta : 1.0f) * (v - m)) * invZ;
          if (top_mask) {
            // a list entry never filled (only with NaN log-joints) reads state 0
            const int64_t ids = (id >= 0 && (int64_t)id < nstates) ? id : 0;
            if (TSC) {
              top_mask[(n * topk + t) * 2 + 0] = tab_act[ids];
              top_mask[(n * topk + t) * 2 + 1] = tab_sgn[ids];
            } else {
              top_mask[n * topk + t] = tab_act[ids];
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
  }
}

// ----------------------------------------------------------------- dispatch
// Shapes with a compile-time tree walk (one tree_*.hip file each).
#define PROSPER_TREE_SHAPES(X) \
  X(false, 12, 4)              \
  X(false, 8, 3)               \
  X(false, 10, 4)              \
  X(false, 12, 5)              \
  X(true, 8, 3)

#define X(T, HP, GM)                                                                      \
  hipError_t launch_tree_##T##_##HP##_##GM(const Prepared&, const Scratch&, int64_t, int,  \
                                           float*, float*, double*, int, float*, int64_t, \
                                           hipStream_t);
PROSPER_TREE_SHAPES(X)
#undef X

bool has_tree_kernel(int model, int Hp, int gamma) {
#define X(T, HP, GM) \
  if ((model == PROSPER_TSC) == T && (model == PROSPER_BSC || model == PROSPER_TSC) && \
      Hp == HP && gamma == GM)                                                            \
    return true;
  PROSPER_TREE_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_states_lin(int model, int Hp, int gamma, int64_t N, int H, int64_t nstates,
                             const uint32_t* tab_act, const uint32_t* tab_sgn,
                             const Prepared& p, const Scratch& s, float* logL,
                             uint32_t* top_mask, float* top_q, int topk, bool acc,
                             float* acc_B, double* scal, int num_cu, int* tree_blocks,
                             hipStream_t st, float beta, float* k_out, float* res_out) {
  if (tree_blocks) *tree_blocks = 0;
  if (N <= 0) return hipSuccess;
  const bool tsc = (model == PROSPER_TSC);
  const bool per_point = k_out || res_out;
  if (topk == 0 && beta == 1.0f && !per_point && has_tree_kernel(model, Hp, gamma)) {
    // training: B partials inside the walk when B's packed triangle fits in LDS
    int nblk = 0;
    if (acc && (int64_t)H * (H + 1) / 2 <= stats_bslice_floats()) {
      int64_t want = (N + 511) / 512;
      nblk = (int)(want < num_cu ? want : num_cu);
      if (tree_blocks) *tree_blocks = nblk;
    }
    float* ss_out = (acc && nblk == 0) ? s.ss : nullptr;
    hipError_t e = hipErrorInvalidValue;
#define X(T, HP, GM)                                                                           \
  if (tsc == T && Hp == HP && gamma == GM)                                                     \
    e = launch_tree_##T##_##HP##_##GM(p, s, N, H, logL, ss_out, scal, nblk, s.partB,           \
                                      (int64_t)stats_bslice_floats(), st);
    PROSPER_TREE_SHAPES(X)
#undef X
    if (e != hipSuccess) return e;
    // points whose weights could overflow with the cheap pivot: exact kernel
    if (gamma > 2) {
      float* Bat = acc ? acc_B : nullptr;
      if (tsc)
        hipLaunchKernelGGL(k_states_generic<true>, dim3(32), dim3(256), 0, st, s.sel, s.bc, s.yy,
                           p.G, H, N, Hp, nstates, tab_act, tab_sgn, p.theta, s.s_mean, logL,
                           top_mask, top_q, 0, (float*)nullptr, Bat, scal, s.redo_list,
                           s.redo_count, (float*)nullptr, (float*)nullptr);
      else
        hipLaunchKernelGGL(k_states_generic<false>, dim3(32), dim3(256), 0, st, s.sel, s.bc,
                           s.yy, p.G, H, N, Hp, nstates, tab_act, tab_sgn, p.theta, s.s_mean,
                           logL, top_mask, top_q, 0, (float*)nullptr, Bat, scal, s.redo_list,
                           s.redo_count, (float*)nullptr, (float*)nullptr);
    }
    return hipGetLastError();
  }
  float* ss_out = acc ? s.ss : nullptr;
  int64_t blocks = (N + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (tsc)
    hipLaunchKernelGGL(k_states_generic<true>, dim3((unsigned)blocks), dim3(256), 0, st, s.sel,
                       s.bc, s.yy, p.G, H, N, Hp, nstates, tab_act, tab_sgn, p.theta, s.s_mean,
                       logL, top_mask, top_q, topk, ss_out, (float*)nullptr, scal, nullptr,
                       nullptr, k_out, res_out);
  else
    hipLaunchKernelGGL(k_states_generic<false>, dim3((unsigned)blocks), dim3(256), 0, st, s.sel,
                       s.bc, s.yy, p.G, H, N, Hp, nstates, tab_act, tab_sgn, p.theta, s.s_mean,
                       logL, top_mask, top_q, topk, ss_out, (float*)nullptr, scal, nullptr,
                       nullptr, k_out, res_out);
  return hipGetLastError();
}

}  // namespace prosper
