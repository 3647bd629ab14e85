// M-step in FP64 on the device (row a9).
//
// BSC / TSC: the joint maximiser of sum_n sum_s q_n(s) log p(y_n, s | Theta):
//   W_new = A B^-1 on the latents with B_hh > 0 (other columns keep W_old),
//   pi_new = sum <k> / (N H),
//   sigma_new^2 = (sum ||y||^2 - tr(W_new^T A)) / (N D),
// the last because W_new B = A on the active block, so that
//   sum_n sum_s q ||y - W_new s||^2 = sum||y||^2 - 2 tr(W^T A) + tr(W^T W B)
// collapses to sum||y||^2 - tr(W_new^T A).
// B arrives as the upper triangle accumulated by the E-step; inactive rows
// and columns are replaced by the identity so that one Cholesky factor
// covers the active block.  A failed pivot restarts the factorisation with a
// diagonal jitter of 1e-10 tr(B)/H (x10 per retry); the attempt count is
// kept in the workspace status word.
// MCA: W_new = A / B elementwise where B > 0 (hard-max responsibilities),
// pi as above, sigma^2 = sum <||y - f(s)||^2> / (N D).
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

struct MstepHdr {
  double trace_WA;  // tr(W_new^T A)
  double jitter;
  int attempts;
  int failed;
};

__global__ __launch_bounds__(1024) void k_mstep_chol(int H, const float* __restrict__ Bup,
                                                     double* __restrict__ L,
                                                     MstepHdr* __restrict__ hdr) {
  __shared__ double piv;
  __shared__ int bad;
  __shared__ double trB;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double t = 0.0;
    for (int h = 0; h < H; ++h) t += (double)Bup[(int64_t)h * H + h];
    trB = t;
    hdr->trace_WA = 0.0;
    hdr->failed = 0;
  }
  __syncthreads();
  double jitter = 0.0;
  for (int attempt = 0; attempt < 4; ++attempt) {
    for (int64_t e = tid; e < (int64_t)H * H; e += nt) {
      const int i = (int)(e / H), j = (int)(e % H);
      const double bii = Bup[(int64_t)i * H + i], bjj = Bup[(int64_t)j * H + j];
      double v;
      if (bii > 0.0 && bjj > 0.0) v = (i <= j) ? (double)Bup[(int64_t)i * H + j] : (double)Bup[(int64_t)j * H + i];
      else v = (i == j) ? 1.0 : 0.0;
      if (i == j && bii > 0.0) v += jitter;
      L[e] = v;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < H; ++k) {
      if (tid == 0) {
        const double d = L[(int64_t)k * H + k];
        if (!(d > 0.0)) {
          bad = 1;
          piv = 1.0;
        } else {
          piv = sqrt(d);
        }
        L[(int64_t)k * H + k] = piv;
      }
      __syncthreads();
      if (bad) break;
      const double inv = 1.0 / piv;
      for (int i = k + 1 + tid; i < H; i += nt) L[(int64_t)i * H + k] *= inv;
      __syncthreads();
      const int m = H - k - 1;
      for (int64_t e = tid; e < (int64_t)m * m; e += nt) {
        const int i = k + 1 + (int)(e / m), j = k + 1 + (int)(e % m);
        if (j <= i) L[(int64_t)i * H + j] -= L[(int64_t)i * H + k] * L[(int64_t)j * H + k];
      }
      __syncthreads();
    }
    if (!bad) {
      if (tid == 0) {
        hdr->attempts = attempt + 1;
        hdr->jitter = jitter;
      }
      return;
    }
    jitter = 1e-10 * pow(10.0, (double)attempt) * (trB > 0.0 ? trB / H : 1.0);
    __syncthreads();
  }
  if (tid == 0) {
    hdr->attempts = 4;
    hdr->failed = 1;
  }
}

// One thread per pixel d: solve L L^T x = A[d, :]^T (active latents), write
// W_new[d, :] and accumulate tr(W_new^T A).
__global__ __launch_bounds__(64) void k_mstep_solve(int D, int H, const float* __restrict__ A,
                                                    const float* __restrict__ Bup,
                                                    const double* __restrict__ L,
                                                    double* __restrict__ X,
                                                    const float* __restrict__ W_old,
                                                    float* __restrict__ W_new,
                                                    MstepHdr* __restrict__ hdr) {
  const int d = blockIdx.x * 64 + threadIdx.x;
  double tr = 0.0;
  if (d < D && !hdr->failed) {
    for (int h = 0; h < H; ++h) {  // forward: L z = a
      const bool act = Bup[(int64_t)h * H + h] > 0.0f;
      double z = act ? (double)A[(int64_t)d * H + h] : 0.0;
      for (int g = 0; g < h; ++g) z -= L[(int64_t)h * H + g] * X[(int64_t)g * D + d];
      X[(int64_t)h * D + d] = z / L[(int64_t)h * H + h];
    }
    for (int h = H - 1; h >= 0; --h) {  // backward: L^T x = z
      double x = X[(int64_t)h * D + d];
      for (int g = h + 1; g < H; ++g) x -= L[(int64_t)g * H + h] * X[(int64_t)g * D + d];
      x /= L[(int64_t)h * H + h];
      X[(int64_t)h * D + d] = x;
    }
    for (int h = 0; h < H; ++h) {
      const bool act = Bup[(int64_t)h * H + h] > 0.0f;
      const double x = X[(int64_t)h * D + d];
      const float a = A[(int64_t)d * H + h];
      if (act) tr += x * (double)a;
      W_new[(int64_t)d * H + h] = act ? (float)x : W_old[(int64_t)d * H + h];
    }
  }
  if (d < D && hdr->failed) {  // keep the old dictionary when no factor was found
    for (int h = 0; h < H; ++h) W_new[(int64_t)d * H + h] = W_old[(int64_t)d * H + h];
  }
  tr = wave_sum_d(tr);
  if (threadIdx.x == 0) atomicAdd(&hdr->trace_WA, tr);
}

__global__ void k_mstep_scalars_lin(int D, int H, const double* __restrict__ scal,
                                    const MstepHdr* __restrict__ hdr,
                                    double* __restrict__ theta_new,
                                    const double* __restrict__ theta_old) {
  if (threadIdx.x || blockIdx.x) return;
  const double N = scal[4];
  const double pi = scal[0] / (N * H);
  const double s2 = (scal[2] - hdr->trace_WA) / (N * D);
  if (hdr->failed) {
    theta_new[0] = theta_old ? theta_old[0] : pi;
    theta_new[1] = theta_old ? theta_old[1] : sqrt(fmax(s2, 0.0));
    return;
  }
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
  hipLaunchKernelGGL(k_mstep_chol, dim3(1), dim3(1024), 0, st, H, B, L, hdr);
  hipLaunchKernelGGL(k_mstep_solve, dim3((D + 63) / 64), dim3(64), 0, st, D, H, A, B, L, X, W_old,
                     W_new, hdr);
  hipLaunchKernelGGL(k_mstep_scalars_lin, dim3(1), dim3(64), 0, st, D, H, scal, hdr, theta_new,
                     (const double*)nullptr);
  return hipGetLastError();
}

}  // namespace prosper
