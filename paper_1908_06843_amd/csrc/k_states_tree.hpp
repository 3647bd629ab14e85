// Compile-time unrolled state walk for linear superposition (BSC, TSC).
//
// One lane per data point.  The truncated state set of (H', gamma) is the
// subset tree whose children of a node add one slot larger than the node's
// last slot; walking it depth first, every state's log-joint (relative to
// the zero state, log2 units) follows from its parent's by one addition:
//   lj(S + j) = lj(S) + w_S[j],   w_S[j] = u_j + sum_{i in S} p_ij
//   w_{S+j}[k] = w_S[k] + p_jk                       (k > j)
// with u_j = c1 + lam (2 b_j - G_jj), p_ij = -2 lam G_ij (BSC).  TSC carries
// signs: lj(S + (j,+-)) = lj(S) + u^+-_j +- v_S[j], v_S[j] = sum_{i in S} s_i p_ij.
// All slot indices are template constants, so u, p, the per-depth w vectors
// and the moment accumulators live in registers.
//
// The walk forms T(node) = sum of 2^(lj - m) over
// the node's subtree; since a state contains slot j exactly when the path
// to it passes the node where j was added:
//   sum_s 2^(lj-m) s_j       = sum over nodes ending in j of T(node)
//   sum_s 2^(lj-m) s_i s_j   = sum over nodes ending in j containing i of T(node)
#pragma once

#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Hide a value's provenance from the optimiser (emits no instruction).  Used
// to keep the pivot walk's values from being reused by the main walk, and to
// pin each accumulator update at its place in the walk: otherwise the backend
// sinks whole accumulation chains to their final use and keeps every
// contribution alive until then.
__device__ __forceinline__ void opaque(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(int& x) { asm volatile("" : "+v"(x)); }

// --------------------------------------------------------------------- BSC
template <int HP, int GAMMA, unsigned PRE, int LAST, int DEPTH>
struct BscTree {
  static __device__ __forceinline__ void walk1(const float (&p)[HP][HP], const float (&w)[HP],
                                               float L, float& mx) {
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      __builtin_amdgcn_sched_barrier(0);
      const float Lc = L + w[j];
      mx = fmaxf(mx, Lc);
      opaque(mx);  // keep the running max a chain (no reassociation into a tree)
      if constexpr (DEPTH + 1 < GAMMA && j + 1 < HP) {
        float wc[HP];
        static_for<j + 1, HP>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          wc[k] = w[k] + p[j][k];
        });
        BscTree<HP, GAMMA, PRE | (1u << j), j, DEPTH + 1>::walk1(p, wc, Lc, mx);
      }
    });
  }
  // returns the summed weight of the children subtrees
  static __device__ __forceinline__ float walk2(const float (&p)[HP][HP], const float (&w)[HP],
                                                float L, float m, float (&M)[HP],
                                                float (&P)[HP][HP]) {
    float tot = 0.0f;
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      __builtin_amdgcn_sched_barrier(0);
      const float Lc = L + w[j];
      float T = fast_exp2(Lc - m);
      if constexpr (DEPTH + 1 < GAMMA && j + 1 < HP) {
        float wc[HP];
        static_for<j + 1, HP>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          wc[k] = w[k] + p[j][k];
        });
        T += BscTree<HP, GAMMA, PRE | (1u << j), j, DEPTH + 1>::walk2(p, wc, Lc, m, M, P);
      }
      M[j] += T;
      opaque(M[j]);
      static_for<0, j>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr ((PRE >> i) & 1u) {
          P[i][j] += T;
          opaque(P[i][j]);
        }
      });
      tot += T;
    });
    return tot;
  }
};

// --------------------------------------------------------------------- TSC
// SGN: minus-sign mask of the prefix.  v[j] = sum_{i in PRE} s_i p_ij.
template <int HP, int GAMMA, unsigned PRE, unsigned SGN, int LAST, int DEPTH>
struct TscTree {
  template <int J, bool NEG>
  static __device__ __forceinline__ void child1(const float (&up)[HP], const float (&um)[HP],
                                                const float (&p)[HP][HP], const float (&v)[HP],
                                                float L, float& mx) {
    __builtin_amdgcn_sched_barrier(0);
    const float Lc = NEG ? L + (um[J] - v[J]) : L + (up[J] + v[J]);
    mx = fmaxf(mx, Lc);
    opaque(mx);
    if constexpr (DEPTH + 1 < GAMMA && J + 1 < HP) {
      float vc[HP];
      static_for<J + 1, HP>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        vc[k] = NEG ? v[k] - p[J][k] : v[k] + p[J][k];
      });
      TscTree<HP, GAMMA, PRE | (1u << J), SGN | (NEG ? (1u << J) : 0u), J, DEPTH + 1>::walk1(
          up, um, p, vc, Lc, mx);
    }
  }
  static __device__ __forceinline__ void walk1(const float (&up)[HP], const float (&um)[HP],
                                               const float (&p)[HP][HP], const float (&v)[HP],
                                               float L, float& mx) {
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      child1<j, false>(up, um, p, v, L, mx);
      child1<j, true>(up, um, p, v, L, mx);
    });
  }
  template <int J, bool NEG>
  static __device__ __forceinline__ float child2(const float (&up)[HP], const float (&um)[HP],
                                                 const float (&p)[HP][HP], const float (&v)[HP],
                                                 float L, float m, float (&M)[HP],
                                                 float (&K2)[HP], float (&P)[HP][HP]) {
    __builtin_amdgcn_sched_barrier(0);
    const float Lc = NEG ? L + (um[J] - v[J]) : L + (up[J] + v[J]);
    float T = fast_exp2(Lc - m);
    if constexpr (DEPTH + 1 < GAMMA && J + 1 < HP) {
      float vc[HP];
      static_for<J + 1, HP>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        vc[k] = NEG ? v[k] - p[J][k] : v[k] + p[J][k];
      });
      T += TscTree<HP, GAMMA, PRE | (1u << J), SGN | (NEG ? (1u << J) : 0u), J,
                   DEPTH + 1>::walk2(up, um, p, vc, Lc, m, M, K2, P);
    }
    if constexpr (NEG) M[J] -= T;
    else M[J] += T;
    K2[J] += T;
    opaque(M[J]);
    opaque(K2[J]);
    static_for<0, J>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr ((PRE >> i) & 1u) {
        constexpr bool ineg = (SGN >> i) & 1u;
        if constexpr (ineg != NEG) P[i][J] -= T;
        else P[i][J] += T;
        opaque(P[i][J]);
      }
    });
    return T;
  }
  static __device__ __forceinline__ float walk2(const float (&up)[HP], const float (&um)[HP],
                                                const float (&p)[HP][HP], const float (&v)[HP],
                                                float L, float m, float (&M)[HP],
                                                float (&K2)[HP], float (&P)[HP][HP]) {
    float tot = 0.0f;
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      tot += child2<j, false>(up, um, p, v, L, m, M, K2, P);
      tot += child2<j, true>(up, um, p, v, L, m, M, K2, P);
    });
    return tot;
  }
};

// Everything one lane does for one data point: the walk and its per-point
// results.  `ok` is false for a point handed to the exact kernel (and for
// lanes without a point).
template <int HP, int GAMMA, bool TSC>
struct PointResult {
  float M[HP], K2[HP], P[HP][HP];
  int s[HP];
  float invZ, kmean;
  double lL;
  bool ok;
};

template <int HP, int GAMMA, bool TSC>
__device__ __forceinline__ void tree_point(PointResult<HP, GAMMA, TSC>& R, int64_t n, bool live,
                                           const int32_t* __restrict__ sel,
                                           const float* __restrict__ bc,
                                           const float* __restrict__ yy,
                                           const float* __restrict__ G, int H, int64_t N,
                                           const Theta* __restrict__ th,
                                           int32_t* __restrict__ redo_list,
                                           int32_t* __restrict__ redo_count) {
  const int64_t nn = live ? n : N - 1;
  const float lam2 = th->lam2, c1 = th->c1_2;
  int* s = R.s;
  float (&M)[HP] = R.M;
  float (&K2)[HP] = R.K2;
  float (&P)[HP][HP] = R.P;
  float b[HP];
#pragma unroll
  for (int j = 0; j < HP; ++j) {
    s[j] = sel[nn * HP + j];
    b[j] = bc[nn * HP + j];
  }
  float p[HP][HP];
#pragma unroll
  for (int i = 0; i < HP; ++i)
#pragma unroll
    for (int j = i + 1; j < HP; ++j) p[i][j] = -2.0f * lam2 * G[(int64_t)s[i] * H + s[j]];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    M[i] = 0.0f;
    K2[i] = 0.0f;
#pragma unroll
    for (int j = i + 1; j < HP; ++j) P[i][j] = 0.0f;
  }
  float m = 0.0f, Z;  // the zero state has lj = 0
  // Pivot m for the weights 2^(lj - m): the max over the states with at most
  // two active slots.  It bounds the max from below, so the weights of those
  // states are <= 1 and Z >= 1, and it saves a second walk for the exact
  // max.  If a deeper state exceeds it by so much that a weight may have
  // overflowed (Z >= 2^64) the point is handed to the exact two-pass kernel
  // through the redo list.  The moments do not depend on the pivot.
  constexpr int GPIV = GAMMA < 2 ? GAMMA : 2;
  if constexpr (!TSC) {
    float u[HP];
#pragma unroll
    for (int j = 0; j < HP; ++j)
      u[j] = c1 + lam2 * (2.0f * b[j] - G[(int64_t)s[j] * H + s[j]]);
    BscTree<HP, GPIV, 0u, -1, 0>::walk1(p, u, 0.0f, m);
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      opaque(u[i]);
#pragma unroll
      for (int j = i + 1; j < HP; ++j) opaque(p[i][j]);
    }
    Z = fast_exp2(-m) + BscTree<HP, GAMMA, 0u, -1, 0>::walk2(p, u, 0.0f, m, M, P);
#pragma unroll
    for (int j = 0; j < HP; ++j) K2[j] = M[j];
  } else {
    float up[HP], um[HP], v0[HP];
#pragma unroll
    for (int j = 0; j < HP; ++j) {
      const float g = G[(int64_t)s[j] * H + s[j]];
      up[j] = c1 + lam2 * (2.0f * b[j] - g);
      um[j] = c1 + lam2 * (-2.0f * b[j] - g);
      v0[j] = 0.0f;
    }
    TscTree<HP, GPIV, 0u, 0u, -1, 0>::walk1(up, um, p, v0, 0.0f, m);
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      opaque(up[i]);
      opaque(um[i]);
      opaque(v0[i]);
#pragma unroll
      for (int j = i + 1; j < HP; ++j) opaque(p[i][j]);
    }
    Z = fast_exp2(-m) + TscTree<HP, GAMMA, 0u, 0u, -1, 0>::walk2(up, um, p, v0, 0.0f, m, M, K2, P);
  }
  R.ok = live;
  if (GAMMA > 2 && live && !(Z < 1.8446744e19f)) {
    R.ok = false;
    const int slot = atomicAdd(redo_count, 1);
    redo_list[slot] = (int32_t)n;
  }
  // fresh copies of the latent indices (keeps the G-gather offsets from being
  // held across the walk for reuse after it)
#pragma unroll
  for (int j = 0; j < HP; ++j) opaque(s[j]);
  R.invZ = 1.0f / Z;
  R.lL = th->c0 - (double)th->lam * (double)yy[nn] +
         0.6931471805599453 * ((double)m + (double)log2f(Z));
  float km = 0.0f;
#pragma unroll
  for (int j = 0; j < HP; ++j) km += K2[j];
  R.kmean = km * R.invZ;
}

// One lane per point, 64-lane workgroups; optional pair-major <s s^T>.
template <int HP, int GAMMA, bool TSC>
__global__ __launch_bounds__(64) void k_states_tree(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, const Theta* __restrict__ th,
    float* __restrict__ s_mean, float* __restrict__ logL, float* __restrict__ ss_out,
    double* __restrict__ scal, int32_t* __restrict__ redo_list, int32_t* __restrict__ redo_count) {
  const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool live = n < N;
  PointResult<HP, GAMMA, TSC> R;
  tree_point<HP, GAMMA, TSC>(R, n, live, sel, bc, yy, G, H, N, th, redo_list, redo_count);
  if (R.ok) {
    if (logL) logL[n] = (float)R.lL;
#pragma unroll
    for (int j = 0; j < HP; ++j) s_mean[n * HP + j] = R.M[j] * R.invZ;
    if (ss_out) {  // pair-major: diagonal first, then i < j row-major
      int q = HP;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        ss_out[(int64_t)i * N + n] = R.K2[i] * R.invZ;
#pragma unroll
        for (int j = i + 1; j < HP; ++j) ss_out[(int64_t)(q++) * N + n] = R.P[i][j] * R.invZ;
      }
    }
  } else if (live && ss_out) {
    // handed to the exact kernel, which adds this point's block to B itself
#pragma unroll
    for (int q = 0; q < HP * (HP + 1) / 2; ++q) ss_out[(int64_t)q * N + n] = 0.0f;
  }
  if (scal) {
    double a0 = R.ok ? (double)R.kmean : 0.0, a1 = R.ok ? R.lL : 0.0;
    a0 = wave_sum_d(a0);
    a1 = wave_sum_d(a1);
    if (threadIdx.x == 0) {
      atomicAdd(&scal[0], a0);
      atomicAdd(&scal[1], a1);
    }
  }
}

// Training variant: persistent 512-lane workgroups (8 waves, the occupancy the
// walk's registers allow anyway) that also add every point's <s s^T> block
// into a workgroup-private copy of B's packed upper triangle in LDS, then
// store that partial with plain stores (partB[block]); the partials are
// summed by the statistics reduction.  Requires H (H + 1) / 2 <= BSLICE floats.
// The LDS copy is fixed point: every term <s_i s_j> lies in [-1, 1] and a
// workgroup adds at most `ppw` of them per entry, so with the quantum
// 1/qscale, qscale = 2^k and ppw 2^k < 2^30, the int32 sums cannot overflow;
// each term is rounded to within 2^-(k+1) (about 5e-7 at k = 20, below the
// terms' own FP32 rounding relative to the sums they enter).  Integer LDS
// atomics run at plain-LDS speed where FP32 LDS atomics do not.
template <int HP, int GAMMA, bool TSC>
__global__ __launch_bounds__(512) void k_states_tree_acc(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, const Theta* __restrict__ th,
    float* __restrict__ s_mean, float* __restrict__ logL, float* __restrict__ partB,
    int64_t part_stride, double* __restrict__ scal, int32_t* __restrict__ redo_list,
    int32_t* __restrict__ redo_count, float qscale) {
  extern __shared__ int Bl[];  // packed upper triangle, row h at h H - h (h - 1) / 2
  __shared__ double red[2][8];
  const int len = H * (H + 1) / 2;
  for (int e = threadIdx.x; e < len; e += 512) Bl[e] = 0;
  __syncthreads();
  double a0 = 0.0, a1 = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * 512; base < N; base += (int64_t)gridDim.x * 512) {
    const int64_t n = base + threadIdx.x;
    const bool live = n < N;
    PointResult<HP, GAMMA, TSC> R;
    tree_point<HP, GAMMA, TSC>(R, n, live, sel, bc, yy, G, H, N, th, redo_list, redo_count);
    if (R.ok) {
      if (logL) logL[n] = (float)R.lL;
#pragma unroll
      for (int j = 0; j < HP; ++j) s_mean[n * HP + j] = R.M[j] * R.invZ;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        const int hi = R.s[i];
        const int row = hi * H - hi * (hi - 1) / 2 - hi;  // packed index of (hi, h2) = row + h2
        atomicAdd(&Bl[row + hi], __float2int_rn(R.K2[i] * R.invZ * qscale));
#pragma unroll
        for (int j = i + 1; j < HP; ++j)
          atomicAdd(&Bl[row + R.s[j]], __float2int_rn(R.P[i][j] * R.invZ * qscale));
      }
      a0 += (double)R.kmean;
      a1 += R.lL;
    }
  }
  __syncthreads();
  float* out = partB + (int64_t)blockIdx.x * part_stride;
  const double unq = 1.0 / (double)qscale;
  for (int e = threadIdx.x; e < len; e += 512) out[e] = (float)((double)Bl[e] * unq);
  if (scal) {
    a0 = wave_sum_d(a0);
    a1 = wave_sum_d(a1);
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = a0;
      red[1][threadIdx.x >> 6] = a1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < 8; ++w) {
        t0 += red[0][w];
        t1 += red[1][w];
      }
      atomicAdd(&scal[0], t0);
      atomicAdd(&scal[1], t1);
    }
  }
}

// Defines the launchers of one compile-time shape: acc_blocks = 0 runs the
// plain kernel; otherwise the training variant on acc_blocks workgroups.
#define PROSPER_TREE_INSTANCE(TSCV, HPV, GMV)                                                    \
  hipError_t launch_tree_##TSCV##_##HPV##_##GMV(const Prepared& p, const Scratch& s, int64_t N,  \
                                                int H, float* logL, float* ss_out, double* scal, \
                                                int acc_blocks, float* partB, int64_t stride,    \
                                                hipStream_t st) {                                \
    if (acc_blocks > 0) {                                                                        \
      /* fixed-point quantum: at most ppw points per workgroup, ppw 2^k < 2^30 */                \
      const int64_t ppw = (N + (int64_t)acc_blocks * 512 - 1) / ((int64_t)acc_blocks * 512) * 512; \
      int k = 0;                                                                                 \
      while (k < 30 && ((int64_t)ppw << (k + 1)) < ((int64_t)1 << 30)) ++k;                     \
      const float qscale = (float)((int64_t)1 << k);                                             \
      auto kern = k_states_tree_acc<HPV, GMV, TSCV>;                                             \
      const size_t lds = (size_t)H * (H + 1) / 2 * 4;                                            \
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);              \
      if (e != hipSuccess) return e;                                                             \
      hipLaunchKernelGGL(kern, dim3((unsigned)acc_blocks), dim3(512), lds, st, s.sel, s.bc,      \
                         s.yy, p.G, H, N, p.theta, s.s_mean, logL, partB, stride, scal,          \
                         s.redo_list, s.redo_count, qscale);                                     \
      return hipGetLastError();                                                                  \
    }                                                                                            \
    hipLaunchKernelGGL((k_states_tree<HPV, GMV, TSCV>), dim3((unsigned)((N + 63) / 64)),         \
                       dim3(64), 0, st, s.sel, s.bc, s.yy, p.G, H, N, p.theta, s.s_mean, logL,   \
                       ss_out, scal, s.redo_list, s.redo_count);                                 \
    return hipGetLastError();                                                                    \
  }

}  // namespace prosper
