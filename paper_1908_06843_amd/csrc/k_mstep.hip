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
// Solve: X = B^-1 A^T (H x D) by a blocked Cholesky factorisation B = L L^T
// (panels of 64 columns) and blocked forward / backward substitution, all
// in FP64.  B arrives as the upper triangle accumulated by the E-step;
// inactive rows and columns are replaced by the identity so one factor
// covers the active block.  A diagonal jitter of 1e-12 tr(B)/H on the active
// diagonal guards the factorisation against round-off at the PSD boundary
// (its effect on W is ~1e-12 relative).  A non-positive pivot is recorded in
// the workspace header and leaves W unchanged.
//   k_ms_panel : one wave factors the 64 x 64 diagonal block in registers
//                (lane i holds row i; column values move by readlane), then
//                the workgroup solves the rows below against it;
//   k_ms_syrk  : trailing update T -= P P^T on 32 x 32 tiles;
//   k_ms_*_diag / k_ms_upd : triangular solves of the diagonal blocks (one
//                thread per right-hand side) and the GEMM updates between.
// MCA: W_new = A / B elementwise where B > 0 (hard-max responsibilities),
// pi as above, sigma^2 = sum <||y - f(s)||^2> / (N D).
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

static constexpr int NB = 64;

struct MstepHdr {
  double trace_WA;  // tr(W_new^T A)
  double trB;       // trace of B (active part)
  int failed;       // a pivot was not positive
  int pad;
};

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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
    hdr->trace_WA = 0.0;
    hdr->failed = 0;
  }
}

__global__ __launch_bounds__(256) void k_ms_load(int D, int H, const float* __restrict__ A,
                                                 const float* __restrict__ Bup,
                                                 const MstepHdr* __restrict__ hdr,
                                                 double* __restrict__ L, double* __restrict__ X) {
  const double jitter = 1e-12 * (hdr->trB > 0.0 ? hdr->trB / H : 1.0);
  const int64_t HH = (int64_t)H * H, HD = (int64_t)H * D;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < HH + HD;
       e += (int64_t)gridDim.x * 256) {
    if (e < HH) {
      const int i = (int)(e / H), j = (int)(e % H);
      const bool ai = Bup[(int64_t)i * H + i] > 0.0f, aj = Bup[(int64_t)j * H + j] > 0.0f;
      double v;
      if (ai && aj) v = (i <= j) ? (double)Bup[(int64_t)i * H + j] : (double)Bup[(int64_t)j * H + i];
      else v = (i == j) ? 1.0 : 0.0;
      if (i == j && ai) v += jitter;
      L[e] = v;
    } else {
      const int64_t f = e - HH;
      const int h = (int)(f / D), d = (int)(f % D);
      const bool ah = Bup[(int64_t)h * H + h] > 0.0f;
      X[f] = ah ? (double)A[(int64_t)d * H + h] : 0.0;
    }
  }
}

// Factor the diagonal block at kb (nb = min(64, H - kb) columns) and solve
// the panel rows below it: L[i, kb:kb+nb] = L[i, kb:kb+nb] L_kk^-T.
__global__ __launch_bounds__(256) void k_ms_panel(int H, int kb, double* __restrict__ L,
                                                  MstepHdr* __restrict__ hdr) {
  __shared__ double Ls[NB][NB + 1];
  const int nb = min(NB, H - kb);
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      a[c] = (lane < nb && c < nb) ? L[(int64_t)(kb + lane) * H + kb + c] : (c == lane ? 1.0 : 0.0);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const double dkk = readlane_d(a[k], k);
      bad |= !(dkk > 0.0);
      const double piv = sqrt(dkk > 0.0 ? dkk : 1.0);
      const double inv = 1.0 / piv;
      a[k] = (lane == k) ? piv : (lane > k ? a[k] * inv : a[k]);
#pragma unroll
      for (int j = k + 1; j < NB; ++j) {
        const double ljk = readlane_d(a[k], j);
        if (lane >= j) a[j] = fma(-a[k], ljk, a[j]);
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) Ls[lane][c] = (c <= lane) ? a[c] : 0.0;
    if (lane < nb) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c <= lane) L[(int64_t)(kb + lane) * H + kb + c] = a[c];
    }
    if (bad && lane == 0) hdr->failed = 1;
  }
  __syncthreads();
  for (int i = kb + nb + tid; i < H; i += 256) {
    double x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = (c < nb) ? L[(int64_t)i * H + kb + c] : 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double v = x[c];
#pragma unroll
      for (int c2 = 0; c2 < c; ++c2) v = fma(-x[c2], Ls[c][c2], v);
      x[c] = v / Ls[c][c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) L[(int64_t)i * H + kb + c] = x[c];
  }
}

// Trailing update for rows/cols >= k1 = kb + nb: T[i][j] -= sum_c P[i][c] P[j][c]
// on 32 x 32 tiles with i-tile >= j-tile.
__global__ __launch_bounds__(256) void k_ms_syrk(int H, int kb, double* __restrict__ L) {
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
  for (int e = threadIdx.x; e < 32 * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Pi[r][c] = (i0 + r < H && c < nb) ? L[(int64_t)(i0 + r) * H + kb + c] : 0.0;
    Pj[r][c] = (j0 + r < H && c < nb) ? L[(int64_t)(j0 + r) * H + kb + c] : 0.0;
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
    L[(int64_t)i * H + j] -= acc;
  }
}

// Forward substitution on the diagonal block: one thread per column d.
__global__ __launch_bounds__(64) void k_ms_fwd_diag(int H, int D, int kb,
                                                    const double* __restrict__ L,
                                                    double* __restrict__ X) {
  const int d = blockIdx.x * 64 + threadIdx.x;
  if (d >= D) return;
  const int nb = min(NB, H - kb);
  double z[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) z[c] = (c < nb) ? X[(int64_t)(kb + c) * D + d] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nb) {
      double v = z[c];
#pragma unroll
      for (int c2 = 0; c2 < c; ++c2) v = fma(-L[(int64_t)(kb + c) * H + kb + c2], z[c2], v);
      z[c] = v / L[(int64_t)(kb + c) * H + kb + c];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < nb) X[(int64_t)(kb + c) * D + d] = z[c];
}

// Backward substitution L_kk^T x = z on the diagonal block.
__global__ __launch_bounds__(64) void k_ms_bwd_diag(int H, int D, int kb,
                                                    const double* __restrict__ L,
                                                    double* __restrict__ X) {
  const int d = blockIdx.x * 64 + threadIdx.x;
  if (d >= D) return;
  const int nb = min(NB, H - kb);
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = (c < nb) ? X[(int64_t)(kb + c) * D + d] : 0.0;
#pragma unroll
  for (int c = NB - 1; c >= 0; --c) {
    if (c < nb) {
      double v = x[c];
#pragma unroll
      for (int c2 = c + 1; c2 < NB; ++c2)
        if (c2 < nb) v = fma(-L[(int64_t)(kb + c2) * H + kb + c], x[c2], v);
      x[c] = v / L[(int64_t)(kb + c) * H + kb + c];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < nb) X[(int64_t)(kb + c) * D + d] = x[c];
}

// X[i][:] -= sum_c M(i, c) X[kb + c][:] for the rows i of [r0, r1):
// forward: M(i, c) = L[i][kb + c] (rows below), backward: M(i, c) = L[kb + c][i] (rows above).
template <bool BWD>
__global__ __launch_bounds__(256) void k_ms_upd(int H, int D, int kb, int r0, int r1,
                                                const double* __restrict__ L,
                                                double* __restrict__ X) {
  __shared__ double Ms[32][NB + 1];
  __shared__ double Xs[NB][65];
  const int nb = min(NB, H - kb);
  const int i0 = r0 + 32 * blockIdx.y, d0 = 64 * blockIdx.x;
  for (int e = threadIdx.x; e < 32 * NB; e += 256) {
    const int r = e / NB, c = e % NB, i = i0 + r;
    double v = 0.0;
    if (i < r1 && c < nb) v = BWD ? L[(int64_t)(kb + c) * H + i] : L[(int64_t)i * H + kb + c];
    Ms[r][c] = v;
  }
  for (int e = threadIdx.x; e < NB * 64; e += 256) {
    const int c = e / 64, dd = e % 64;
    Xs[c][dd] = (c < nb && d0 + dd < D) ? X[(int64_t)(kb + c) * D + d0 + dd] : 0.0;
  }
  __syncthreads();
  const int dd = threadIdx.x & 63, rb = (threadIdx.x >> 6) * 8;
  if (d0 + dd >= D) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = rb + q, i = i0 + r;
    if (i >= r1) break;
    double acc = 0.0;
#pragma unroll 8
    for (int c = 0; c < NB; ++c) acc = fma(Ms[r][c], Xs[c][dd], acc);
    X[(int64_t)i * D + d0 + dd] -= acc;
  }
}

// W_new and tr(W_new^T A).
__global__ __launch_bounds__(256) void k_ms_finish(int D, int H, const float* __restrict__ A,
                                                   const float* __restrict__ Bup,
                                                   const double* __restrict__ X,
                                                   const float* __restrict__ W_old,
                                                   float* __restrict__ W_new,
                                                   MstepHdr* __restrict__ hdr) {
  __shared__ double red[4];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double tr = 0.0;
  const bool ok = !hdr->failed;
  if (e < (int64_t)D * H) {
    const int d = (int)(e / H), h = (int)(e % H);
    const bool act = Bup[(int64_t)h * H + h] > 0.0f;
    if (ok && act) {
      const double x = X[(int64_t)h * D + d];
      tr = x * (double)A[e];
      W_new[e] = (float)x;
    } else {
      W_new[e] = W_old[e];
    }
  }
  tr = wave_sum_d(tr);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tr;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&hdr->trace_WA, red[0] + red[1] + red[2] + red[3]);
}

__global__ void k_ms_scalars_lin(int D, int H, const double* __restrict__ scal,
                                 const MstepHdr* __restrict__ hdr, double* __restrict__ theta_new) {
  if (threadIdx.x || blockIdx.x) return;
  const double N = scal[4];
  const double pi = scal[0] / (N * H);
  const double s2 = (scal[2] - hdr->trace_WA) / (N * D);
  theta_new[0] = pi;
  theta_new[1] = sqrt(fmax(s2, 0.0));
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
  if (model == PROSPER_MCA) return 256;
  return 256 + (size_t)H * H * 8 + (size_t)H * D * 8;
}

hipError_t launch_mstep(int model, int D, int H, const float* A, const float* B,
                        const double* scal, const float* W_old, float* W_new,
                        double* theta_new, void* work, hipStream_t st) {
  if (model == PROSPER_MCA) {
    const int64_t n = (int64_t)D * H;
    hipLaunchKernelGGL(k_mstep_mca, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, H, A,
                       B, W_old, W_new);
    hipLaunchKernelGGL(k_mstep_scalars_mca, dim3(1), dim3(64), 0, st, D, H, scal, theta_new);
    return hipGetLastError();
  }
  MstepHdr* hdr = reinterpret_cast<MstepHdr*>(work);
  double* L = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + 256);
  double* X = L + (size_t)H * H;
  hipLaunchKernelGGL(k_ms_begin, dim3(1), dim3(1024), 0, st, H, B, hdr);
  const int64_t nload = (int64_t)H * H + (int64_t)H * D;
  int64_t lb = (nload + 255) / 256;
  if (lb > 2048) lb = 2048;
  hipLaunchKernelGGL(k_ms_load, dim3((unsigned)lb), dim3(256), 0, st, D, H, A, B, hdr, L, X);
  for (int kb = 0; kb < H; kb += NB) {
    hipLaunchKernelGGL(k_ms_panel, dim3(1), dim3(256), 0, st, H, kb, L, hdr);
    const int k1 = kb + NB;
    if (k1 < H) {
      const int nt = (H - k1 + 31) / 32;
      hipLaunchKernelGGL(k_ms_syrk, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, H, kb,
                         L);
    }
  }
  const dim3 gdiag((D + 63) / 64);
  for (int kb = 0; kb < H; kb += NB) {
    hipLaunchKernelGGL(k_ms_fwd_diag, gdiag, dim3(64), 0, st, H, D, kb, L, X);
    const int r0 = kb + NB;
    if (r0 < H)
      hipLaunchKernelGGL(k_ms_upd<false>, dim3((D + 63) / 64, (H - r0 + 31) / 32), dim3(256), 0,
                         st, H, D, kb, r0, H, L, X);
  }
  const int last = ((H - 1) / NB) * NB;
  for (int kb = last; kb >= 0; kb -= NB) {
    hipLaunchKernelGGL(k_ms_bwd_diag, gdiag, dim3(64), 0, st, H, D, kb, L, X);
    if (kb > 0)
      hipLaunchKernelGGL(k_ms_upd<true>, dim3((D + 63) / 64, (kb + 31) / 32), dim3(256), 0, st,
                         H, D, kb, 0, kb, L, X);
  }
  const int64_t n = (int64_t)D * H;
  hipLaunchKernelGGL(k_ms_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, H, A,
                     B, X, W_old, W_new, hdr);
  hipLaunchKernelGGL(k_ms_scalars_lin, dim3(1), dim3(64), 0, st, D, H, scal, hdr, theta_new);
  return hipGetLastError();
}

}  // namespace prosper
