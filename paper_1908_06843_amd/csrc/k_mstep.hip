// M-step in FP64 on the device (row a9).
//
// BSC / TSC: the joint maximiser of sum_n sum_s q_n(s) log p(y_n, s | Theta):
//   W_new = A B^-1 on the latents with B_hh > 0 (other columns keep W_old),
//   pi_new = sum <k> / (N H),
//   sigma_new^2 = (sum ||y||^2 - tr(W_new^T A)) / (N D),
// the last because W_new B = A on the active block, so that
//   sum_n sum_s q ||y - W_new s||^2 = sum||y||^2 - 2 tr(W^T A) + tr(W^T W B)
// collapses to sum||y||^2 - tr(W_new^T A).
//
// Solve: row d of W_new is x = B^-1 a_d (a_d = row d of A) on the active
// block.  B arrives as the upper triangle accumulated by the E-step; inactive
// rows and columns are replaced by the identity so one factor covers the
// active block.  A diagonal jitter of 1e-12 tr(B)/H on the active diagonal
// guards the factorisation against round-off at the PSD boundary (its effect
// on W is ~1e-12 relative).  A non-positive pivot is recorded in the
// workspace header and leaves W unchanged.
//   k_ms_panel : right-looking blocked Cholesky B = L L^T with 64-column
//                panels.  Every workgroup factors the 64 x 64 diagonal block
//                in one wave's registers (lane i holds row i), then solves 256
//                of the rows below it.  The factor is written twice: L in the
//                lower triangle and L^T in the upper one, so that both
//                triangular solves read contiguous rows;
//   k_ms_syrk  : trailing update T -= P P^T on 32 x 32 tiles;
//   k_ms_solve : one wave per pixel d: forward and backward substitution of
//                x with its 64-row blocks in registers (lane i holds x[64 m + i]);
//                the 64 x 64 blocks of L are staged in LDS one step ahead,
//                shared by the workgroup's four pixels; then W_new row d and
//                its share of tr(W_new^T A).
// MCA: W_new = A / B elementwise where B > 0 (hard-max responsibilities),
// pi as above, sigma^2 = sum <||y - f(s)||^2> / (N D).
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

static constexpr int NB = 64;

struct MstepHdr {
  double trB;  // trace of B (active part)
  int failed;  // a pivot was not positive
  int pad;
};

// Workspace: header | M (H x H) | invd (H) | trp (D), each 256-byte aligned.
struct MstepWork {
  MstepHdr* hdr;
  double* M;
  double* invd;
  double* trp;
};

static MstepWork carve_mstep(void* work, int D, int H) {
  char* p = reinterpret_cast<char*>(work);
  MstepWork w;
  w.hdr = reinterpret_cast<MstepHdr*>(p);
  p += 256;
  w.M = reinterpret_cast<double*>(p);
  p += round_up((size_t)H * H * 8, 256);
  w.invd = reinterpret_cast<double*>(p);
  p += round_up((size_t)H * 8, 256);
  w.trp = reinterpret_cast<double*>(p);
  return w;
}

__global__ __launch_bounds__(1024) void k_ms_begin(int H, const float* __restrict__ Bup,
                                                   MstepHdr* __restrict__ hdr) {
  __shared__ double red[16];
  double t = 0.0;
  for (int h = threadIdx.x; h < H; h += 1024) {
    const float b = Bup[(int64_t)h * H + h];
    if (b > 0.0f) t += (double)b;
  }
  t = wave_sum_d(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += red[w];
    hdr->trB = s;
    hdr->failed = 0;
  }
}

// M = symmetrised active block of B (+ jitter), identity on inactive latents.
__global__ __launch_bounds__(256) void k_ms_load(int H, const float* __restrict__ Bup,
                                                 const MstepHdr* __restrict__ hdr,
                                                 double* __restrict__ M) {
  const double jitter = 1e-12 * (hdr->trB > 0.0 ? hdr->trB / H : 1.0);
  const int64_t HH = (int64_t)H * H;
  // unconditional loads (upper-triangle element, both diagonals) so that
  // the unrolled iterations keep their loads in flight together
#pragma unroll 4
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < HH;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / H), j = (int)(e % H);
    const float bii = Bup[(int64_t)i * H + i], bjj = Bup[(int64_t)j * H + j];
    const float bu = Bup[(int64_t)min(i, j) * H + max(i, j)];
    const bool ai = bii > 0.0f, aj = bjj > 0.0f;
    double v = (ai && aj) ? (double)bu : ((i == j) ? 1.0 : 0.0);
    if (i == j && ai) v += jitter;
    M[e] = v;
  }
}

__device__ __forceinline__ double rsqrt_refined(double d) {
  const double r = __builtin_amdgcn_rsq(d);
  return r * fma(-0.5 * d * r, r, 1.5);
}

// Right-looking Cholesky of a diagonal block held one row per lane
// (a[c] = element (lane, c)).  Column k is scaled by the pivot's reciprocal
// square root and then broadcast through the wave's LDS buffer col.  Rows
// above the pivot are updated too: their entries form the upper triangle,
// which is never read, and skipping the selects halves the work.
template <int NBK>
__device__ __forceinline__ void factor_rows(double (&a)[NBK], int lane, double* col,
                                            double& myinv, bool& bad) {
  static_for<0, NBK>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    __builtin_amdgcn_sched_barrier(0);
    const double dkk = readlane_d(a[k], k);
    bad |= !(dkk > 0.0);
    const double dpos = dkk > 0.0 ? dkk : 1.0;
    const double inv = rsqrt_refined(dpos);
    myinv = (lane == k) ? inv : myinv;
    a[k] = (lane == k) ? dpos * inv : a[k] * inv;
    if (lane < NBK) col[lane] = a[k];
    static_for<k + 1, NBK>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      a[j] = fma(-a[k], col[j], a[j]);
    });
  });
  __builtin_amdgcn_sched_barrier(0);
}

// Panel at kb (nb = min(64, H - kb) columns): factor the diagonal block,
// then L[i, kb:kb+nb] = M[i, kb:kb+nb] L_kk^-T for the 256 rows of this
// workgroup's share of i >= kb + nb.  Each workgroup factors the (small)
// diagonal block itself; workgroup 0 writes it back with its mirror and
// the inverse pivots.
__global__ __launch_bounds__(256) void k_ms_panel(int H, int kb, double* __restrict__ M,
                                                  double* __restrict__ invd,
                                                  MstepHdr* __restrict__ hdr) {
  __shared__ double Ls[NB][NB + 1];  // transposed: Ls[c][r] = L[r][c]
  __shared__ double inv_s[NB];
  __shared__ double colb[NB];
  const int nb = min(NB, H - kb);
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    // lane i holds row kb + i of the block; padding rows/columns are the
    // identity.  Addresses are clamped so every load is unconditional.
    const double* rp = M + (int64_t)min(kb + lane, H - 1) * H + kb;
    double a[NB];
    static_for<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const double v = rp[c < nb ? c : 0];
      a[c] = (lane < nb && c < nb) ? v : (c == lane ? 1.0 : 0.0);
    });
    bool bad = false;
    double myinv = 1.0;
    factor_rows<NB>(a, lane, colb, myinv, bad);
    static_for<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      Ls[c][lane] = (c <= lane) ? a[c] : 0.0;
    });
    inv_s[lane] = myinv;
    if (blockIdx.x == 0 && bad && lane == 0) hdr->failed = 1;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    // write the factored block and its mirror, and the inverse pivots
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (r < nb && c <= r) {
        const double v = Ls[c][r];
        M[(int64_t)(kb + r) * H + kb + c] = v;
        M[(int64_t)(kb + c) * H + kb + r] = v;
      }
    }
    if (tid < nb) invd[kb + tid] = inv_s[tid];
  }
  // rows below the block exist only when the block is full (nb == 64)
  const int i = kb + nb + blockIdx.x * 256 + tid;
  if (i >= H) return;
  double* xp = M + (int64_t)i * H + kb;
  double x[NB];
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    x[c] = xp[c];
  });
  // right-looking: x_c /= L_cc, then x_c' -= x_c L_c'c for c' > c
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    // one scheduling region per step: otherwise every LDS read of the block
    // is hoisted to the top and the registers spill
    __builtin_amdgcn_sched_barrier(0);
    x[c] = x[c] * inv_s[c];
    static_for<c + 1, NB>([&](auto c2c) {
      constexpr int c2 = decltype(c2c)::value;
      x[c2] = fma(-x[c], Ls[c][c2], x[c2]);
    });
  });
  __builtin_amdgcn_sched_barrier(0);
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    xp[c] = x[c];
    M[(int64_t)(kb + c) * H + i] = x[c];
  });
}

// Trailing update for rows/cols >= k1 = kb + nb: T[i][j] -= sum_c P[i][c] P[j][c]
// on 32 x 32 tiles with i-tile >= j-tile (lower triangle only).
__global__ __launch_bounds__(256) void k_ms_syrk(int H, int kb, double* __restrict__ M) {
  __shared__ double Pi[32][NB + 1], Pj[32][NB + 1];
  const int nb = min(NB, H - kb), k1 = kb + nb;
  // blockIdx.x enumerates lower-triangle tile pairs (ti >= tj)
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int i0 = k1 + 32 * ti, j0 = k1 + 32 * tj;
  // every load of the two 32 x 64 panels is issued before the first LDS
  // store (clamped addresses, masked values): this kernel runs beside the
  // HBM-bound statistics, where each dependent round trip costs microseconds
  constexpr int PER = 32 * NB / 256;
  double vi[PER], vj[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    const int r = e / NB, c = e % NB;
    const int cc = c < nb ? c : 0;
    const double a = M[(int64_t)min(i0 + r, H - 1) * H + kb + cc];
    const double b = M[(int64_t)min(j0 + r, H - 1) * H + kb + cc];
    vi[k] = (i0 + r < H && c < nb) ? a : 0.0;
    vj[k] = (j0 + r < H && c < nb) ? b : 0.0;
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    Pi[e / NB][e % NB] = vi[k];
    Pj[e / NB][e % NB] = vj[k];
  }
  __syncthreads();
  const int r = threadIdx.x >> 3, cb = (threadIdx.x & 7) * 4;  // 32 rows x (8 x 4 cols)
  const int i = i0 + r;
  if (i >= H) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jj = cb + q, j = j0 + jj;
    if (j >= H || j > i) continue;
    double acc = 0.0;
#pragma unroll 8
    for (int c = 0; c < NB; ++c) acc = fma(Pi[r][c], Pj[jj][c], acc);
    M[(int64_t)i * H + j] -= acc;
  }
}

// Block steps of the two substitutions on 64-row blocks (compile-time list):
// forward: for each block mb its diagonal solve, then its update of every
// block below; backward: blocks in reverse, diagonal solve, then its update
// of every block above.  Each step reads the 64 x 64 block of M in rows
// 64 mb .. + 64 and columns 64 tgt .. + 64.
struct SolveStep {
  int mb, tgt, kind;  // kind: 0 forward diagonal, 1 forward update, 2 backward diagonal, 3 backward update
};
template <int MB>
struct SolveSteps {
  SolveStep s[MB * (MB + 1)];
  constexpr SolveSteps() : s() {
    int k = 0;
    for (int mb = 0; mb < MB; ++mb) {
      s[k++] = SolveStep{mb, mb, 0};
      for (int m = mb + 1; m < MB; ++m) s[k++] = SolveStep{mb, m, 1};
    }
    for (int mb = MB - 1; mb >= 0; --mb) {
      s[k++] = SolveStep{mb, mb, 2};
      for (int m = 0; m < mb; ++m) s[k++] = SolveStep{mb, m, 3};
    }
  }
};

// x = B^-1 a_d for pixel d = 4 blockIdx.x + wave, H <= 64 MB.  Lane i holds
// x[64 m + i] in x[m].  Uses M[p][q] = L[max(p,q)][min(p,q)]: row kb + c of
// M holds column kb + c of L to the right of the diagonal and row kb + c of
// L to its left.  The M block of each step is staged in LDS by the whole
// workgroup (shared by its four pixels) one step ahead of its use.  Writes
// row d of W_new and the wave's part of tr(W_new^T A).
template <int MB>
__global__ __launch_bounds__(256) void k_ms_solve(int D, int H, const float* __restrict__ A,
                                                  const float* __restrict__ Bup,
                                                  const double* __restrict__ M,
                                                  const double* __restrict__ invd,
                                                  const MstepHdr* __restrict__ hdr,
                                                  const float* W_old, float* W_new,
                                                  double* __restrict__ trp) {
  constexpr SolveSteps<MB> steps{};
  constexpr int NS = MB * (MB + 1);
  __shared__ double Ms[2][64][64];
  __shared__ double Is[2][64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int d = blockIdx.x * 4 + (tid >> 6);
  const bool dok = d < D;
  const int64_t row = (int64_t)(dok ? d : 0) * H;
  const bool failed = hdr->failed != 0;
  double x[MB];
  bool act[MB];
  static_for<0, MB>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    const int h = 64 * m + lane;
    act[m] = h < H && Bup[(int64_t)(h < H ? h : 0) * H + (h < H ? h : 0)] > 0.0f;
    const float a = A[row + (h < H ? h : 0)];
    x[m] = act[m] ? (double)a : 0.0;
  });
  // staged block of a step: element (c, i) = M[kb + c][64 tgt + i] (zero
  // outside H).  Diagonal blocks are staged pre-multiplied by the inverse
  // pivot of row c and with the already-final side of the triangle zeroed,
  // so the substitution is one fma per column and every lane scales its own
  // value at the end.  Global loads run two steps ahead (two register sets),
  // the LDS copy one step ahead (two buffers).
  double reg[2][16];
  double ireg[2] = {0.0, 0.0};
  auto load_block = [&](int set, int mb, int tgt, int kind) {
    const int kb = 64 * mb, cb = 64 * tgt;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, c = e >> 6, i = e & 63;
      bool ok = kb + c < H && cb + i < H;
      if (kind == 0) ok = ok && i > c;
      if (kind == 2) ok = ok && i < c;
      const double v = M[(int64_t)(ok ? kb + c : 0) * H + (ok ? cb + i : 0)];
      double sc = 1.0;
      if (kind == 0 || kind == 2) sc = invd[kb + c < H ? kb + c : 0];
      reg[set][u] = ok ? v * sc : 0.0;
    }
    if (tid < 64) {
      const double v = invd[kb + tid < H ? kb + tid : 0];
      ireg[set] = kb + tid < H ? v : 0.0;
    }
  };
  auto store_block = [&](int set, int buf) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      Ms[buf][e >> 6][e & 63] = reg[set][u];
    }
    if (tid < 64) Is[buf][tid] = ireg[set];
  };
  auto step_live = [&](const SolveStep& st) { return 64 * st.mb < H && 64 * st.tgt < H; };
  load_block(0, steps.s[0].mb, steps.s[0].tgt, steps.s[0].kind);
  // loads are unconditional (clamped addresses) so that the waits before the
  // LDS copies count only the older loads
  if constexpr (NS > 1) load_block(1, steps.s[1].mb, steps.s[1].tgt, steps.s[1].kind);
  store_block(0, 0);
  __syncthreads();
  static_for<0, NS>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr SolveStep st = steps.s[k];
    constexpr int buf = k & 1;
    const int kb = 64 * st.mb;
    if constexpr (k + 2 < NS) {
      constexpr SolveStep n2 = steps.s[k + 2];
      load_block(k & 1, n2.mb, n2.tgt, n2.kind);
    }
    if (step_live(st)) {
      const int nb = min(64, H - kb);
      if constexpr (st.kind == 0) {
        // v_i -= (L_ic / L_cc) v_c for i > c; then x_i = v_i / L_ii
#pragma unroll 16
        for (int c = 0; c < nb; ++c)
          x[st.mb] = fma(-Ms[buf][c][lane], readlane_d(x[st.mb], c), x[st.mb]);
        x[st.mb] *= Is[buf][lane];
      } else if constexpr (st.kind == 2) {
#pragma unroll 16
        for (int c = nb - 1; c >= 0; --c)
          x[st.mb] = fma(-Ms[buf][c][lane], readlane_d(x[st.mb], c), x[st.mb]);
        x[st.mb] *= Is[buf][lane];
      } else {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
        for (int c = 0; c + 1 < nb; c += 2) {
          a0 = fma(Ms[buf][c][lane], readlane_d(x[st.mb], c), a0);
          a1 = fma(Ms[buf][c + 1][lane], readlane_d(x[st.mb], c + 1), a1);
        }
        if (nb & 1) a0 = fma(Ms[buf][nb - 1][lane], readlane_d(x[st.mb], nb - 1), a0);
        x[st.tgt] -= a0 + a1;
      }
    }
    if constexpr (k + 1 < NS) {
      store_block((k + 1) & 1, buf ^ 1);
      __syncthreads();
    }
  });
  if (!dok) return;
  if (failed) {
    for (int h = lane; h < H; h += 64) W_new[row + h] = W_old[row + h];
    if (lane == 0) trp[d] = 0.0;
    return;
  }
  double tr = 0.0;
  static_for<0, MB>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    const int h = 64 * m + lane;
    if (h < H) {
      if (act[m]) {
        tr = fma(x[m], (double)A[row + h], tr);
        W_new[row + h] = (float)x[m];
      } else {
        W_new[row + h] = W_old[row + h];
      }
    }
  });
  tr = wave_sum_d(tr);
  if (lane == 0) trp[d] = tr;
}

__global__ __launch_bounds__(256) void k_ms_scalars_lin(int D, int H,
                                                        const double* __restrict__ scal,
                                                        const double* __restrict__ trp,
                                                        double* __restrict__ theta_new) {
  __shared__ double red[4];
  double t = 0.0;
  for (int d = threadIdx.x; d < D; d += 256) t += trp[d];
  t = wave_sum_d(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double trace_WA = red[0] + red[1] + red[2] + red[3];
    const double N = scal[4];
    theta_new[0] = scal[0] / (N * H);
    const double s2 = (scal[2] - trace_WA) / (N * D);
    theta_new[1] = sqrt(fmax(s2, 0.0));
  }
}

__global__ __launch_bounds__(256) void k_mstep_mca(int D, int H, const float* __restrict__ A,
                                                   const float* __restrict__ B,
                                                   const float* __restrict__ W_old,
                                                   float* __restrict__ W_new) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)D * H) return;
  const float b = B[e];
  W_new[e] = (b > 0.0f) ? (float)((double)A[e] / (double)b) : W_old[e];
}

__global__ void k_mstep_scalars_mca(int D, int H, const double* __restrict__ scal,
                                    double* __restrict__ theta_new) {
  if (threadIdx.x || blockIdx.x) return;
  const double N = scal[4];
  theta_new[0] = scal[0] / (N * H);
  theta_new[1] = sqrt(fmax(scal[3] / (N * D), 0.0));
}

size_t mstep_workspace_bytes(int model, int D, int H) {
  if (is_max_model(model)) return 256;
  return 256 + round_up((size_t)H * H * 8, 256) + round_up((size_t)H * 8, 256) +
         round_up((size_t)D * 8, 256);
}

template <int MB>
static void launch_solve(int D, int H, const float* A, const float* B, const MstepWork& w,
                         const float* W_old, float* W_new, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_solve<MB>, dim3((unsigned)((D + 3) / 4)), dim3(256), 0, st, D, H, A, B,
                     w.M, w.invd, w.hdr, W_old, W_new, w.trp);
}

hipError_t launch_mstep_factor(int model, int D, int H, const float* B, void* work,
                               hipStream_t st) {
  if (is_max_model(model)) return hipSuccess;
  if (H > 16 * 64) return hipErrorInvalidValue;
  const MstepWork w = carve_mstep(work, D, H);
  hipLaunchKernelGGL(k_ms_begin, dim3(1), dim3(1024), 0, st, H, B, w.hdr);
  const int64_t HH = (int64_t)H * H;
  // at most 16 workgroups: when B is factored beside the A statistics only
  // the CUs those leave out are free, and more workgroups than fit there
  // wait for the statistics to end
  int64_t lb = (HH + 2047) / 2048;
  if (lb > 16) lb = 16;
  hipLaunchKernelGGL(k_ms_load, dim3((unsigned)lb), dim3(256), 0, st, H, B, w.hdr, w.M);
  for (int kb = 0; kb < H; kb += NB) {
    const int nb = (H - kb < NB) ? H - kb : NB;
    const int below = H - kb - nb;
    const unsigned nblk = below > 0 ? (unsigned)((below + 255) / 256) : 1u;
    hipLaunchKernelGGL(k_ms_panel, dim3(nblk), dim3(256), 0, st, H, kb, w.M, w.invd, w.hdr);
    if (below > 0) {
      const int nt = (below + 31) / 32;
      hipLaunchKernelGGL(k_ms_syrk, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, H, kb,
                         w.M);
    }
  }
  return hipGetLastError();
}

hipError_t launch_mstep_solve(int model, int D, int H, const float* A, const float* B,
                              const double* scal, const float* W_old, float* W_new,
                              double* theta_new, void* work, hipStream_t st) {
  if (is_max_model(model)) {
    const int64_t n = (int64_t)D * H;
    hipLaunchKernelGGL(k_mstep_mca, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, H, A,
                       B, W_old, W_new);
    hipLaunchKernelGGL(k_mstep_scalars_mca, dim3(1), dim3(64), 0, st, D, H, scal, theta_new);
    return hipGetLastError();
  }
  if (H > 16 * 64) return hipErrorInvalidValue;
  const MstepWork w = carve_mstep(work, D, H);
  if (H <= 64) launch_solve<1>(D, H, A, B, w, W_old, W_new, st);
  else if (H <= 128) launch_solve<2>(D, H, A, B, w, W_old, W_new, st);
  else if (H <= 256) launch_solve<4>(D, H, A, B, w, W_old, W_new, st);
  else if (H <= 512) launch_solve<8>(D, H, A, B, w, W_old, W_new, st);
  else launch_solve<16>(D, H, A, B, w, W_old, W_new, st);
  hipLaunchKernelGGL(k_ms_scalars_lin, dim3(1), dim3(256), 0, st, D, H, scal, w.trp, theta_new);
  return hipGetLastError();
}

hipError_t launch_mstep(int model, int D, int H, const float* A, const float* B,
                        const double* scal, const float* W_old, float* W_new,
                        double* theta_new, void* work, hipStream_t st) {
  hipError_t e = launch_mstep_factor(model, D, H, B, work, st);
  if (e != hipSuccess) return e;
  return launch_mstep_solve(model, D, H, A, B, scal, W_old, W_new, theta_new, work, st);
}

}  // namespace prosper
