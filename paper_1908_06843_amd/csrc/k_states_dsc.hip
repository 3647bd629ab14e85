// State walk for discrete sparse coding (DSC: latents take one of V values
// phi_0 = 0, phi_1, ..., phi_{V-1} with a categorical prior, linear
// superposition and Gaussian noise; Table 1).
//
// Relative to the zero state and in log2 units the log-joint of a state of
// K_n with actives j (slots of the preselection, c_j = I_n(j)) at values
// v_j splits into singleton and pair terms of the candidates, as for BSC
// and TSC, now with the value of each active entering both:
//   lj(s) = sum_j u_{v_j}(j) + sum_{j<j'} phi_{v_j} phi_{v_j'} g(j, j'),
//   u_v(j) = log2(pv_v/pv_0) + lam2 (2 phi_v b_cj - phi_v^2 G_cjcj),
//   g(j, j') = -2 lam2 G_cjcj'
// (Eq. 1 categorical prior, Eq. 2 with f = W s; b = W^T y, G = W^T W).
//
// One wave per data point, lanes stride over the state table (act: active
// slot mask; code: the 3-bit value codes of the actives, lowest slot first).
// Pass 1 finds the maximum and the lanes' top lists, pass 2 accumulates the
// weights per (value, slot) and per slot pair in LDS; the moments follow:
//   <s_j> = sum_v phi_v Q_v(j) / Z,  <s_j^2> = sum_v phi_v^2 Q_v(j) / Z,
//   <#latents at phi_v> = sum_j Q_v(j) / Z,  <s_j s_j'> = P(j, j') / Z.
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

namespace {

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

struct DscLds {
  float u[DSC_MAXV][32];  // singleton terms per value (row 0 unused)
  float g[32 * 32];       // pair base terms, i < j
  float Q[DSC_MAXV][32];  // weight of the states with slot j at value v
  float P[32 * 32];       // sum of weight * phi_i phi_j, i < j
  float phi[DSC_MAXV];
};

// Log-joint (relative, log2) of one state from the LDS terms.
__device__ __forceinline__ float dsc_state_lj(const DscLds& S, uint32_t act, uint32_t code) {
  float L = 0.0f;
  uint32_t rem = act, cw = code;
  while (rem) {
    const int j = __ffs(rem) - 1;
    rem &= rem - 1u;
    const int cj = (int)(cw & 7u);
    cw >>= 3;
    L += S.u[cj][j];
    const float pj = S.phi[cj];
    uint32_t pre = act & ((1u << j) - 1u), ci_w = code;
    while (pre) {
      const int i = __ffs(pre) - 1;
      pre &= pre - 1u;
      const int ci = (int)(ci_w & 7u);
      ci_w >>= 3;
      L += (S.phi[ci] * pj) * S.g[i * 32 + j];
    }
  }
  return L;
}

}  // namespace

__global__ __launch_bounds__(256) void k_states_dsc(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, int Hp, int64_t nstates,
    const uint32_t* __restrict__ tab_act, const uint32_t* __restrict__ tab_code,
    const Theta* __restrict__ th, float* __restrict__ s_mean, float* __restrict__ logL,
    uint32_t* __restrict__ top_mask, float* __restrict__ top_q, int topk,
    float* __restrict__ ss_out, double* __restrict__ vcount, double* __restrict__ scal,
    const int32_t* __restrict__ list, const int32_t* __restrict__ list_count,
    float* __restrict__ B_atomic) {
  __shared__ DscLds sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  DscLds& S = sh[wave];
  const float lam2 = th->lam2;
  const int nv = th->nv;
  const float beta = th->beta;
  const bool tempered = beta != 1.0f;
  double acc_k = 0.0, acc_l = 0.0, acc_v = 0.0;  // acc_v: value `lane` (1 <= lane < nv)
  // list mode: only the points named in list[0 .. *list_count)
  const int64_t npts = list ? (int64_t)*list_count : N;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < npts; base += (int64_t)gridDim.x * 4) {
    const bool live = base + wave < npts;
    const int64_t n = !live ? 0 : (list ? (int64_t)list[base + wave] : base + wave);
    if (live) {
      if (lane < DSC_MAXV) S.phi[lane] = lane < nv ? th->phi[lane] : 0.0f;
      for (int j = lane; j < Hp; j += 64) {
        const int sj = sel[n * Hp + j];
        const float gjj = G[(int64_t)sj * H + sj];
        const float bj = bc[n * Hp + j];
        for (int v = 0; v < DSC_MAXV; ++v) {
          const float ph = th->phi[v];
          S.u[v][j] = (v >= 1 && v < nv) ? th->u2[v] + lam2 * (2.0f * ph * bj - ph * ph * gjj)
                                         : 0.0f;
          S.Q[v][j] = 0.0f;
        }
      }
      for (int idx = lane; idx < Hp * Hp; idx += 64) {
        const int i = idx / Hp, j = idx % Hp;
        if (i < j) {
          S.g[i * 32 + j] = -2.0f * lam2 * G[(int64_t)sel[n * Hp + i] * H + sel[n * Hp + j]];
          S.P[i * 32 + j] = 0.0f;
        }
      }
    }
    __syncthreads();
    // pass 1: max and the lane's top list (states visited in increasing index)
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
        const float L = dsc_state_lj(S, tab_act[k], tab_code[k]);
        mx = fmaxf(mx, L);
        if (topk > 0) {
          float v = L;
          int id = (int)k;
#pragma unroll
          for (int t = 0; t < PROSPER_MAX_TOPK; ++t) {
            const bool better = v > tv[t];
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
    // pass 2: weights into the (value, slot) and pair accumulators
    float z = 0.0f, z1 = 0.0f;
    if (live) {
      for (int64_t k = lane; k < nstates; k += 64) {
        const uint32_t act = tab_act[k], code = tab_code[k];
        const float L = dsc_state_lj(S, act, code);
        const float e1 = exp2_fast(L - m);
        const float e = tempered ? exp2_fast(beta * (L - m)) : e1;
        z += e;
        z1 += e1;
        uint32_t rem = act, cw = code;
        while (rem) {
          const int j = __ffs(rem) - 1;
          rem &= rem - 1u;
          const int cj = (int)(cw & 7u);
          cw >>= 3;
          atomicAdd(&S.Q[cj][j], e);
          const float ej = e * S.phi[cj];
          uint32_t pre = act & ((1u << j) - 1u), ci_w = code;
          while (pre) {
            const int i = __ffs(pre) - 1;
            pre &= pre - 1u;
            const int ci = (int)(ci_w & 7u);
            ci_w >>= 3;
            atomicAdd(&S.P[i * 32 + j], ej * S.phi[ci]);
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
      for (int j = lane; j < Hp; j += 64) {
        float m1 = 0.0f, m2 = 0.0f;
        for (int v = 1; v < nv; ++v) {
          const float q = S.Q[v][j];
          m1 += S.phi[v] * q;
          m2 += S.phi[v] * S.phi[v] * q;
        }
        s_mean[n * Hp + j] = m1 * invZ;
        if (ss_out) ss_out[(int64_t)j * N + n] = m2 * invZ;
        if (B_atomic) {
          const int sj = sel[n * Hp + j];
          atomicAdd(&B_atomic[(int64_t)sj * H + sj], m2 * invZ);
        }
      }
      if (B_atomic) {  // few points (the compiled walk's redo list): direct adds
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
            ss_out[(int64_t)p * N + n] = S.P[i * 32 + j] * invZ;
          }
        }
      }
      // expected number of latents at each value: lane v sums Q_v over the slots
      float vm = 0.0f;
      if (lane >= 1 && lane < nv)
        for (int j = 0; j < Hp; ++j) vm += S.Q[lane][j];
      vm *= invZ;
      const float kmean = wave_sum(vm);
      acc_v += vm;
      if (lane == 0) {
        if (logL) logL[n] = (float)lL;
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
          if (top_q) top_q[n * topk + t] = exp2_fast((tempered ? beta : 1.0f) * (v - m)) * invZ;
          if (top_mask) {
            // active mask and the three bit planes of the value codes (a
            // list entry never filled, possible only with NaN log-joints,
            // reads state 0)
            const int64_t ids = (id >= 0 && (int64_t)id < nstates) ? id : 0;
            const uint32_t act = tab_act[ids];
            uint32_t cw = tab_code[ids], rem = act, p0 = 0u, p1 = 0u, p2 = 0u;
            while (rem) {
              const int j = __ffs(rem) - 1;
              rem &= rem - 1u;
              p0 |= (cw & 1u) << j;
              p1 |= ((cw >> 1) & 1u) << j;
              p2 |= ((cw >> 2) & 1u) << j;
              cw >>= 3;
            }
            uint32_t* o = top_mask + (n * topk + t) * 4;
            o[0] = act;
            o[1] = p0;
            o[2] = p1;
            o[3] = p2;
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
  if (vcount && lane >= 1 && lane < nv) atomicAdd(&vcount[lane], acc_v);
}

// ------------------------------------------------------------ compiled walk
// One lane per data point; the subset tree of (H', gamma) unrolled at compile
// time (children of a node add one slot after the node's last slot), the
// values of each added slot a uniform loop over v = 1 .. V-1.  With
// f_S[k] = sum_{i in S} phi_{v_i} p_ik (p_ik = -2 lam2 G_ik), the child
// (S + j at v) has
//   lj = lj(S) + c_v + phi_v (b2_j + f_S[j] - phi_v g_j),   b2_j = 2 lam2 b_j,
//   g_j = lam2 G_jj,  c_v = log2(pv_v/pv_0),
//   f_{S+j}[k] = f_S[k] + phi_v p_jk   (k > j).
// T(node) = the summed weight 2^(lj - m) of the node's subtree; a state holds
// slot j at value v exactly when its path passes the node that added (j, v):
//   Q_v(j) = sum of T over the nodes adding (j, v), <s_j> Z = sum phi_v Q_v(j),
//   <s_j^2> Z = sum phi_v^2 Q_v(j), <s_i s_j> Z = sum over nodes adding (j, v)
//   below an ancestor (i, v_i) of phi_{v_i} phi_v T.
template <int HP>
struct DscCtx {
  float b2[HP], g[HP];
  float p[HP][HP];
  float ph[DSC_MAXV], c[DSC_MAXV];  // value v and its prior constant (compile-time index)
  const Theta* th;                  // the same for a runtime (uniform) index
  int nv;
};

__device__ __forceinline__ void keep(float& x) { asm volatile("" : "+v"(x)); }

// A node at DEPTH whose children are the last level (DEPTH + 1 == GAMMA)
// unrolls the values of its children at compile time (guarded by v < V), so
// every value-indexed operand is a register; the upper levels, a small share
// of the states, loop over the values at run time with scalar loads.
template <int HP, int GAMMA, unsigned PRE, int LAST, int DEPTH>
struct DscTree {
  static constexpr bool LEAVES = DEPTH + 1 >= GAMMA;

  static __device__ __forceinline__ void walk1(const DscCtx<HP>& C, const float (&f)[HP],
                                               float L, float& mx) {
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const float bj = C.b2[j] + f[j];
      if constexpr (LEAVES) {
        static_for<1, DSC_MAXV>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          if (v < C.nv) {
            const float ph = C.ph[v];
            mx = fmaxf(mx, L + (C.c[v] + ph * (bj - ph * C.g[j])));
            keep(mx);
          }
        });
      } else {
        for (int v = 1; v < C.nv; ++v) {
          const float ph = C.th->phi[v];
          const float Lc = L + (C.th->u2[v] + ph * (bj - ph * C.g[j]));
          mx = fmaxf(mx, Lc);
          keep(mx);
          if constexpr (j + 1 < HP) {
            float fc[HP];
            static_for<j + 1, HP>([&](auto kc) {
              constexpr int k = decltype(kc)::value;
              fc[k] = f[k] + ph * C.p[j][k];
            });
            DscTree<HP, GAMMA, PRE | (1u << j), j, DEPTH + 1>::walk1(C, fc, Lc, mx);
          }
        }
      }
    });
  }

  // Moments of the node (j, v) with subtree weight T; aph[d] = value of the
  // prefix's d-th active.
  template <int J>
  static __device__ __forceinline__ void moments(float ph, float T, const float (&aph)[GAMMA + 1],
                                                 float (&M)[HP], float (&K2)[HP],
                                                 float (&P)[HP][HP]) {
    const float pT = ph * T;
    M[J] += pT;
    K2[J] += ph * pT;
    keep(M[J]);
    keep(K2[J]);
    static_for<0, J>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr ((PRE >> i) & 1u) {
        constexpr int d = __builtin_popcount(PRE & ((1u << i) - 1u));
        P[i][J] += aph[d] * pT;
        keep(P[i][J]);
      }
    });
  }

  // returns the summed weight of the children subtrees
  static __device__ __forceinline__ float walk2(const DscCtx<HP>& C, const float (&f)[HP],
                                                const float (&aph)[GAMMA + 1], float L, float m,
                                                float (&M)[HP], float (&K2)[HP],
                                                float (&P)[HP][HP], float (&VC)[DSC_MAXV]) {
    float tot = 0.0f;
    static_for<LAST + 1, HP>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if constexpr (LEAVES) {
        const float bj = C.b2[j] + f[j];
        static_for<1, DSC_MAXV>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          if (v < C.nv) {
            const float ph = C.ph[v];
            const float T = exp2_fast(L + (C.c[v] + ph * (bj - ph * C.g[j])) - m);
            moments<j>(ph, T, aph, M, K2, P);
            VC[v] += T;
            keep(VC[v]);
            tot += T;
          }
        });
      }
    });
    if constexpr (!LEAVES) {
      // values outermost: the children's weights at value v are summed over
      // the slots first, and that sum enters VC[v] by selects (a runtime index
      // into VC would put the array in scratch memory)
      for (int v = 1; v < C.nv; ++v) {
        const float ph = C.th->phi[v], cv = C.th->u2[v];
        float tv = 0.0f;
        static_for<LAST + 1, HP>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const float Lc = L + (cv + ph * ((C.b2[j] + f[j]) - ph * C.g[j]));
          float T = exp2_fast(Lc - m);
          if constexpr (j + 1 < HP) {
            float fc[HP];
            static_for<j + 1, HP>([&](auto kc) {
              constexpr int k = decltype(kc)::value;
              fc[k] = f[k] + ph * C.p[j][k];
            });
            float ac[GAMMA + 1];
            static_for<0, DEPTH>([&](auto dc) {
              constexpr int d = decltype(dc)::value;
              ac[d] = aph[d];
            });
            ac[DEPTH] = ph;
            T += DscTree<HP, GAMMA, PRE | (1u << j), j, DEPTH + 1>::walk2(C, fc, ac, Lc, m, M,
                                                                          K2, P, VC);
          }
          moments<j>(ph, T, aph, M, K2, P);
          tv += T;
        });
        static_for<1, DSC_MAXV>([&](auto vc) {
          constexpr int vv = decltype(vc)::value;
          VC[vv] += (v == vv) ? tv : 0.0f;
          keep(VC[vv]);
        });
        tot += tv;
      }
    }
    return tot;
  }
};

// Everything one lane does for one point of the compiled walk.  Pivot m =
// the max over the states with at most two actives (a lower bound of the
// max: those weights are <= 1 and Z >= 1); a point whose Z could have
// overflowed (>= 2^64) is handed to the table-driven kernel through the redo
// list (ok = false) and written by it.
template <int HP, int GAMMA>
struct DscPoint {
  float M[HP], K2[HP], P[HP][HP], VC[DSC_MAXV];
  int s[HP];
  float invZ;
  double lL;
  bool ok;
};

template <int HP, int GAMMA>
__device__ __forceinline__ void dsc_tree_point(DscPoint<HP, GAMMA>& R, int64_t n, bool live,
                                               const int32_t* __restrict__ sel,
                                               const float* __restrict__ bc,
                                               const float* __restrict__ yy,
                                               const float* __restrict__ G, int H, int64_t N,
                                               const Theta* __restrict__ th,
                                               int32_t* __restrict__ redo_list,
                                               int32_t* __restrict__ redo_count) {
  const int64_t nn = live ? n : N - 1;
  const float lam2 = th->lam2;
  DscCtx<HP> C;
  C.th = th;
  C.nv = th->nv;
#pragma unroll
  for (int v = 0; v < DSC_MAXV; ++v) {
    C.ph[v] = th->phi[v];
    C.c[v] = th->u2[v];
  }
#pragma unroll
  for (int j = 0; j < HP; ++j) {
    R.s[j] = sel[nn * HP + j];
    C.b2[j] = 2.0f * lam2 * bc[nn * HP + j];
    C.g[j] = lam2 * G[(int64_t)R.s[j] * H + R.s[j]];
  }
#pragma unroll
  for (int i = 0; i < HP; ++i)
#pragma unroll
    for (int j = i + 1; j < HP; ++j) C.p[i][j] = -2.0f * lam2 * G[(int64_t)R.s[i] * H + R.s[j]];
  float f0[HP], a0[GAMMA + 1];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    R.M[i] = 0.0f;
    R.K2[i] = 0.0f;
    f0[i] = 0.0f;
#pragma unroll
    for (int j = i + 1; j < HP; ++j) R.P[i][j] = 0.0f;
  }
#pragma unroll
  for (int v = 0; v < DSC_MAXV; ++v) R.VC[v] = 0.0f;
#pragma unroll
  for (int d = 0; d <= GAMMA; ++d) a0[d] = 0.0f;
  float m = 0.0f;  // the zero state has lj = 0
  constexpr int GPIV = GAMMA < 2 ? GAMMA : 2;
  DscTree<HP, GPIV, 0u, -1, 0>::walk1(C, f0, 0.0f, m);
  const float Z = exp2_fast(-m) + DscTree<HP, GAMMA, 0u, -1, 0>::walk2(C, f0, a0, 0.0f, m, R.M,
                                                                        R.K2, R.P, R.VC);
  R.ok = live;
  if (GAMMA > 2 && live && !(Z < 1.8446744e19f)) {
    R.ok = false;
    redo_list[atomicAdd(redo_count, 1)] = (int32_t)n;
  }
  // fresh copies of the latent indices (keeps the G-gather offsets from being
  // held across the walk for reuse after it)
#pragma unroll
  for (int j = 0; j < HP; ++j) asm volatile("" : "+v"(R.s[j]));
  R.invZ = 1.0f / Z;
  R.lL = th->c0 - (double)th->lam * (double)yy[nn] +
         0.6931471805599453 * ((double)m + (double)log2f(Z));
}

// One lane per point, 64-lane workgroups; optional pair-major <s s^T>.
template <int HP, int GAMMA>
__global__ __launch_bounds__(64) void k_states_dsc_tree(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, const Theta* __restrict__ th,
    float* __restrict__ s_mean, float* __restrict__ logL, float* __restrict__ ss_out,
    double* __restrict__ vcount, double* __restrict__ scal, int32_t* __restrict__ redo_list,
    int32_t* __restrict__ redo_count) {
  const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
  DscPoint<HP, GAMMA> R;
  dsc_tree_point<HP, GAMMA>(R, n, n < N, sel, bc, yy, G, H, N, th, redo_list, redo_count);
  const float invZ = R.invZ;
  float km = 0.0f;
  if (R.ok) {
    if (logL) logL[n] = (float)R.lL;
#pragma unroll
    for (int j = 0; j < HP; ++j) s_mean[n * HP + j] = R.M[j] * invZ;
    if (ss_out) {  // pair-major: diagonal first, then i < j row-major
      int q = HP;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        ss_out[(int64_t)i * N + n] = R.K2[i] * invZ;
#pragma unroll
        for (int j = i + 1; j < HP; ++j) ss_out[(int64_t)(q++) * N + n] = R.P[i][j] * invZ;
      }
    }
#pragma unroll
    for (int v = 1; v < DSC_MAXV; ++v) km += R.VC[v];
  }
  if (scal) {
    double k0 = R.ok ? (double)(km * invZ) : 0.0, l0 = R.ok ? R.lL : 0.0;
    k0 = wave_sum_d(k0);
    l0 = wave_sum_d(l0);
    if (threadIdx.x == 0) {
      atomicAdd(&scal[0], k0);
      atomicAdd(&scal[1], l0);
    }
  }
  if (vcount) {
    const int nv = th->nv;
#pragma unroll
    for (int v = 1; v < DSC_MAXV; ++v) {
      if (v < nv) {
        const double t = wave_sum_d(R.ok ? (double)(R.VC[v] * invZ) : 0.0);
        if (threadIdx.x == 0) atomicAdd(&vcount[v], t);
      }
    }
  }
}

// Training variant: persistent 512-lane workgroups that add every point's
// <s s^T> block into a workgroup-private copy of B's packed upper triangle in
// LDS, as int32 fixed point (every term lies within max phi_v^2 in
// magnitude; a workgroup adds at most ppw terms per entry; the quantum
// 1/qscale, qscale = 2^k, keeps ppw max phi^2 2^k below 2^30), then store
// that partial with plain stores (partB[block]) for the statistics reduction.
// Requires H (H + 1) / 2 <= the partial's length.
template <int HP, int GAMMA>
__global__ __launch_bounds__(512) void k_states_dsc_tree_acc(
    const int32_t* __restrict__ sel, const float* __restrict__ bc, const float* __restrict__ yy,
    const float* __restrict__ G, int H, int64_t N, const Theta* __restrict__ th,
    float* __restrict__ s_mean, float* __restrict__ logL, float* __restrict__ partB,
    int64_t part_stride, double* __restrict__ vcount, double* __restrict__ scal,
    int32_t* __restrict__ redo_list, int32_t* __restrict__ redo_count) {
  extern __shared__ int Bq[];  // packed upper triangle, row h at h H - h (h - 1) / 2
  __shared__ double red[2 + DSC_MAXV][8];
  const int len = H * (H + 1) / 2;
  for (int e = threadIdx.x; e < len; e += 512) Bq[e] = 0;
  const int64_t ppw = (N + (int64_t)gridDim.x * 512 - 1) / ((int64_t)gridDim.x * 512) * 512;
  const double bound = (double)ppw * (double)th->phimax * (double)th->phimax;
  int k = 0;
  while (k < 30 && bound * (double)(1ll << (k + 1)) < 1073741824.0) ++k;
  const float qscale = (float)(1ll << k);
  const int nv = th->nv;
  __syncthreads();
  double a0 = 0.0, a1 = 0.0, av[DSC_MAXV];
#pragma unroll
  for (int v = 0; v < DSC_MAXV; ++v) av[v] = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * 512; base < N; base += (int64_t)gridDim.x * 512) {
    const int64_t n = base + threadIdx.x;
    DscPoint<HP, GAMMA> R;
    dsc_tree_point<HP, GAMMA>(R, n, n < N, sel, bc, yy, G, H, N, th, redo_list, redo_count);
    if (R.ok) {
      const float invZ = R.invZ;
      if (logL) logL[n] = (float)R.lL;
#pragma unroll
      for (int j = 0; j < HP; ++j) s_mean[n * HP + j] = R.M[j] * invZ;
      const float qz = invZ * qscale;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        const int hi = R.s[i];
        const int row = hi * H - hi * (hi - 1) / 2 - hi;  // packed index of (hi, h2) = row + h2
        atomicAdd(&Bq[row + hi], __float2int_rn(R.K2[i] * qz));
#pragma unroll
        for (int j = i + 1; j < HP; ++j) atomicAdd(&Bq[row + R.s[j]], __float2int_rn(R.P[i][j] * qz));
      }
      float km = 0.0f;
#pragma unroll
      for (int v = 1; v < DSC_MAXV; ++v) {
        km += R.VC[v];
        av[v] += (double)(R.VC[v] * invZ);
      }
      a0 += (double)(km * invZ);
      a1 += R.lL;
    }
  }
  __syncthreads();
  float* out = partB + (int64_t)blockIdx.x * part_stride;
  const double unq = 1.0 / (double)qscale;
  for (int e = threadIdx.x; e < len; e += 512) out[e] = (float)((double)Bq[e] * unq);
  // FP64 sums of the workgroup: <k>, logL and the value counts
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  a0 = wave_sum_d(a0);
  a1 = wave_sum_d(a1);
  if (lane == 0) {
    red[0][w] = a0;
    red[1][w] = a1;
  }
#pragma unroll
  for (int v = 1; v < DSC_MAXV; ++v) {
    const double t = wave_sum_d(av[v]);
    if (lane == 0) red[2 + v][w] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2 + DSC_MAXV) {
    const int r = threadIdx.x;
    double t = 0.0;
    for (int q = 0; q < 8; ++q) t += red[r][q];
    if (r < 2) {
      if (scal) atomicAdd(&scal[r], t);
    } else if (r >= 3 && r - 2 < nv && vcount) {
      atomicAdd(&vcount[r - 2], t);
    }
  }
}

// Shapes with a compiled DSC walk (any V).
bool has_dsc_tree(int Hp, int gamma) { return Hp == 8 && gamma == 3; }

hipError_t launch_states_dsc(int Hp, int gamma, int64_t N, int H, int64_t nstates,
                             const uint32_t* tab_act, const uint32_t* tab_code, const Prepared& p,
                             const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, bool acc, double* vcount, double* scal, hipStream_t st,
                             float beta, int num_cu, int* tree_blocks, float* acc_B) {
  if (tree_blocks) *tree_blocks = 0;
  if (N <= 0) return hipSuccess;
  double* vc = acc ? vcount : nullptr;
  if (topk == 0 && beta == 1.0f && has_dsc_tree(Hp, gamma)) {
    // training: B partials inside the walk when B's packed triangle fits
    int nblk = 0;
    if (acc && (int64_t)H * (H + 1) / 2 <= stats_bslice_floats()) {
      const int64_t want = (N + 511) / 512;
      nblk = (int)(want < num_cu ? want : num_cu);
      if (tree_blocks) *tree_blocks = nblk;
    }
    if (nblk > 0) {
      auto kern = k_states_dsc_tree_acc<8, 3>;
      const size_t lds = (size_t)H * (H + 1) / 2 * 4;
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(512), lds, st, s.sel, s.bc, s.yy, p.G,
                         H, N, p.theta, s.s_mean, logL, s.partB,
                         (int64_t)stats_bslice_floats(), vc, scal, s.redo_list, s.redo_count);
    } else {
      hipLaunchKernelGGL((k_states_dsc_tree<8, 3>), dim3((unsigned)((N + 63) / 64)), dim3(64), 0,
                         st, s.sel, s.bc, s.yy, p.G, H, N, p.theta, s.s_mean, logL,
                         acc ? s.ss : nullptr, vc, scal, s.redo_list, s.redo_count);
    }
    // points whose weights could overflow with the pivot: the table-driven
    // kernel (with the B partials, their <s s^T> goes straight into acc_B)
    hipLaunchKernelGGL(k_states_dsc, dim3(32), dim3(256), 0, st, s.sel, s.bc, s.yy, p.G, H, N,
                       Hp, nstates, tab_act, tab_code, p.theta, s.s_mean, logL, top_mask, top_q,
                       0, (acc && nblk == 0) ? s.ss : nullptr, vc, scal, s.redo_list,
                       s.redo_count, nblk > 0 ? acc_B : nullptr);
    return hipGetLastError();
  }
  int64_t blocks = (N + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_states_dsc, dim3((unsigned)blocks), dim3(256), 0, st, s.sel, s.bc, s.yy,
                     p.G, H, N, Hp, nstates, tab_act, tab_code, p.theta, s.s_mean, logL,
                     top_mask, top_q, topk, acc ? s.ss : nullptr, vc, scal, nullptr, nullptr,
                     (float*)nullptr);
  return hipGetLastError();
}

}  // namespace prosper
