// Per-call parameter preparation (row a1 of the hot path): derived constants
// of (pi, sigma), the transposed projection matrix in FP32 and as a BF16
// head/tail pair, the Gram matrix G = W^T W and the half squared norms of
// the projection rows.  All reductions are accumulated in FP64 and rounded
// once, so the FP32 state walk starts from correctly rounded G and norms.
#include <cmath>

#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

// pi, sigma from the host values or from device memory (written by the
// M-step); also clears the running max of the projection-row norms, the
// redo-list counter of the unrolled state walk and the counter of points the
// projection hands to the deferred exact selection.
// DSC: the prior pv from the host values or from theta_dev[2 ..], and the
// per-value constants of the walk and of the selection score.
__global__ void k_theta(int model, int D, int H, double pi_h, double sigma_h,
                        const double* __restrict__ theta_dev, Theta* __restrict__ th,
                        float* __restrict__ pnorm, int32_t* __restrict__ redo_count,
                        int32_t* __restrict__ defer_count, float beta, DscParams dsc,
                        double* __restrict__ zscal, double* __restrict__ zvc, int nvc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (zscal)
    for (int i = 0; i < 5; ++i) zscal[i] = 0.0;
  if (zvc)
    for (int v = 0; v < nvc; ++v) zvc[v] = 0.0;
  double pi = theta_dev ? theta_dev[0] : pi_h;
  double sigma = theta_dev ? theta_dev[1] : sigma_h;
  const double LOG2E = 1.4426950408889634;
  Theta t;
  t.sigma = sigma;
  const double lgauss = 0.5 * (double)D * log(2.0 * M_PI * sigma * sigma);
  double lam = 1.0 / (2.0 * sigma * sigma);
  t.lam = (float)lam;
  t.lam2 = (float)(lam * LOG2E);
  t.ln2 = (float)0.6931471805599453;
  t.beta = beta;
  t.nv = 0;
  t.phimax = 0.0f;
  t.csmax = 0.0f;
  for (int v = 0; v < DSC_MAXV; ++v) {
    t.phi[v] = 0.0f;
    t.u2[v] = 0.0f;
    t.cs[v] = 0.0f;
    t.csd[v] = 0.0;
  }
  if (model == PROSPER_DSC) {
    const double p0 = theta_dev ? theta_dev[2] : dsc.pv[0];
    t.nv = dsc.nv;
    pi = 1.0 - p0;
    for (int v = 1; v < dsc.nv; ++v) {
      const double lr = log((theta_dev ? theta_dev[2 + v] : dsc.pv[v]) / p0);
      t.phi[v] = dsc.phi[v];
      t.u2[v] = (float)(lr * LOG2E);
      t.csd[v] = sigma * sigma * lr;
      t.cs[v] = (float)t.csd[v];
      t.phimax = fmaxf(t.phimax, fabsf(dsc.phi[v]));
      t.csmax = fmaxf(t.csmax, fabsf(t.cs[v]));
    }
    t.c0 = (double)H * log(p0) - lgauss;
    t.c1_2 = 0.0f;
  } else {
    t.c0 = (double)H * log1p(-pi) - lgauss;
    double c1 = (model == PROSPER_TSC) ? log(pi / (2.0 * (1.0 - pi))) : log(pi / (1.0 - pi));
    t.c1_2 = (float)(c1 * LOG2E);
  }
  t.pi = pi;
  *th = t;
  *pnorm = 0.0f;
  if (redo_count) *redo_count = 0;
  if (defer_count) *defer_count = 0;
}

// Pt32[h][d] = P[d][h] (zero for d >= D), P = W or max(W, 0) (MCA, H > 1);
// optional BF16 head/tail split.  32 x 32 tiles through LDS.
// zA, zB (optional): D x H accumulators cleared on the way (same index map as W).
__device__ __forceinline__ void transpose_tile(int bx, int by, const float* __restrict__ W, int D,
                                               int H, int Dp, int relu, float* __restrict__ Pt32,
                                               bf16* __restrict__ Pt_hi, bf16* __restrict__ Pt_lo,
                                               float* __restrict__ zA, float* __restrict__ zB) {
  __shared__ float tile[32][33];
  const int d0 = bx * 32, h0 = by * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int d = d0 + r, h = h0 + tx;
    float v = 0.0f;
    if (d < D && h < H) {
      v = W[(int64_t)d * H + h];
      if (relu) v = fmaxf(v, 0.0f);
      if (zA) zA[(int64_t)d * H + h] = 0.0f;
      if (zB) zB[(int64_t)d * H + h] = 0.0f;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int h = h0 + r, d = d0 + tx;
    if (h < H && d < Dp) {
      float v = tile[tx][r];
      int64_t o = (int64_t)h * Dp + d;
      Pt32[o] = v;
      if (Pt_hi) {
        bf16 hi = (bf16)v;
        Pt_hi[o] = hi;
        Pt_lo[o] = (bf16)(v - (float)hi);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ W, int D, int H,
                                                   int Dp, int relu, float* __restrict__ Pt32,
                                                   bf16* __restrict__ Pt_hi,
                                                   bf16* __restrict__ Pt_lo,
                                                   float* __restrict__ zA,
                                                   float* __restrict__ zB) {
  transpose_tile(blockIdx.x, blockIdx.y, W, D, H, Dp, relu, Pt32, Pt_hi, Pt_lo, zA, zB);
}

// G[i][j] = sum_d W[d][i] W[d][j], FP64 accumulation, one 16 x 16 output tile
// per workgroup.  Depth goes in chunks of 256 rows of W: both 16-column slabs
// of a chunk are staged in LDS by one load phase, the four waves take 64 rows
// each (every lane a 2 x 2 block of the tile), and the four partial tiles are
// summed in wave order at the end.  zB (optional): the H x H accumulator
// cleared on the way.  hn_hi (optional): the diagonal also gives
// hn[h] = 1/2 ||W_h||^2 (FP64 head and tail) and the running max of ||W_h||_2,
// as k_norms forms them for P = W.
__device__ __forceinline__ void gram_tile(int bx, int by, const float* __restrict__ W, int D, int H,
                                          float* __restrict__ G, float* __restrict__ zB,
                                          float* __restrict__ hn_hi, float* __restrict__ hn_lo,
                                          float* __restrict__ pnorm) {
  constexpr int KC = 256;
  __shared__ float a[KC][16], b[KC][16];  // a[k][c] = W[d0 + k][i0 + c], b likewise at j0
  __shared__ double part[4][16][16];
  const int i0 = by * 16, j0 = bx * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = (lane >> 3) * 2, c = (lane & 7) * 2;
  double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
  for (int d0 = 0; d0 < D; d0 += KC) {
#pragma unroll
    for (int u = 0; u < KC * 16 / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int k = e >> 4, q = e & 15;
      const int d = d0 + k;
      a[k][q] = (d < D && i0 + q < H) ? W[(int64_t)d * H + i0 + q] : 0.0f;
      b[k][q] = (d < D && j0 + q < H) ? W[(int64_t)d * H + j0 + q] : 0.0f;
    }
    __syncthreads();
    const int k0 = wave * (KC / 4);
#pragma unroll 8
    for (int k = k0; k < k0 + KC / 4; ++k) {
      const float2 av = *reinterpret_cast<const float2*>(&a[k][r]);
      const float2 bv = *reinterpret_cast<const float2*>(&b[k][c]);
      const double a0 = av.x, a1 = av.y, b0 = bv.x, b1 = bv.y;
      acc00 = fma(a0, b0, acc00);
      acc01 = fma(a0, b1, acc01);
      acc10 = fma(a1, b0, acc10);
      acc11 = fma(a1, b1, acc11);
    }
    __syncthreads();
  }
  part[wave][r][c] = acc00;
  part[wave][r][c + 1] = acc01;
  part[wave][r + 1][c] = acc10;
  part[wave][r + 1][c + 1] = acc11;
  __syncthreads();
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const int i = i0 + ti, j = j0 + tj;
  if (i < H && j < H) {
    const double g = ((part[0][ti][tj] + part[1][ti][tj]) + part[2][ti][tj]) + part[3][ti][tj];
    G[(int64_t)i * H + j] = (float)g;
    if (zB) zB[(int64_t)i * H + j] = 0.0f;
    if (hn_hi && i == j) {
      const double half = 0.5 * g;
      const float hi = (float)half;
      hn_hi[i] = hi;
      hn_lo[i] = (float)(half - (double)hi);
      atomicMax(reinterpret_cast<unsigned int*>(pnorm), __float_as_uint((float)sqrt(g)));
    }
  }
}

// Linear models: the transpose and the Gram matrix in one launch (both only
// read W).  Workgroups [0, ntx * nty) take the 32 x 32 transpose tiles, the
// rest the 16 x 16 Gram tiles (ngx per row).
__global__ __launch_bounds__(256) void k_transpose_gram(
    const float* __restrict__ W, int D, int H, int Dp, int ntx, int nty, int ngx,
    float* __restrict__ Pt32, bf16* __restrict__ Pt_hi, bf16* __restrict__ Pt_lo,
    float* __restrict__ zA, float* __restrict__ G, float* __restrict__ zB,
    float* __restrict__ hn_hi, float* __restrict__ hn_lo, float* __restrict__ pnorm) {
  const int nt = ntx * nty;
  const int b = blockIdx.x;
  if (b < nt)
    transpose_tile(b % ntx, b / ntx, W, D, H, Dp, 0, Pt32, Pt_hi, Pt_lo, zA, nullptr);
  else
    gram_tile((b - nt) % ngx, (b - nt) / ngx, W, D, H, G, zB, hn_hi, hn_lo, pnorm);
}

// hn[h] = 1/2 ||P_h||^2 in FP64 split into an FP32 head and tail; running
// max of ||P_h||_2 (positive floats order like their bit patterns).  One
// wave per latent, lanes over pixels of the transposed (contiguous) row.
__global__ __launch_bounds__(256) void k_norms(const float* __restrict__ Pt32, int Dp, int H,
                                               float* __restrict__ hn_hi, float* __restrict__ hn_lo,
                                               float* __restrict__ pnorm) {
  const int h = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (h >= H) return;
  double acc = 0.0;
  for (int d = lane; d < Dp; d += 64) {
    const double v = Pt32[(int64_t)h * Dp + d];
    acc = fma(v, v, acc);
  }
  acc = wave_sum_d(acc);
  if (lane == 0) {
    const double half = 0.5 * acc;
    const float hi = (float)half;
    hn_hi[h] = hi;
    hn_lo[h] = (float)(half - (double)hi);
    atomicMax(reinterpret_cast<unsigned int*>(pnorm), __float_as_uint((float)sqrt(acc)));
  }
}

// wmax[d] = max_h W_dh (unclamped), one thread per pixel over its contiguous row.
__global__ __launch_bounds__(256) void k_rowmax(const float* __restrict__ W, int D, int H,
                                                float* __restrict__ wmax) {
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= D) return;
  float m = -INFINITY;
  for (int h = 0; h < H; ++h) m = fmaxf(m, W[(int64_t)d * H + h]);
  wmax[d] = m;
}

hipError_t launch_prep(int model, int prec, const float* W, int D, int H, int Dp,
                       const Prepared& p, hipStream_t st, const AccZero& z) {
  const int relu = (model == PROSPER_MCA && H > 1) ? 1 : 0;
  dim3 gt((Dp + 31) / 32, (H + 31) / 32);
  bf16* hi = prec != PROSPER_FP32 ? p.Pt_hi : nullptr;
  bf16* lo = prec != PROSPER_FP32 ? p.Pt_lo : nullptr;
  if (!is_max_model(model) && !z.B_dh) {
    // P = W: one launch for the transpose and G; the norms come from G's diagonal
    const int ngx = (H + 15) / 16;
    const unsigned nblk = gt.x * gt.y + (unsigned)(ngx * ngx);
    hipLaunchKernelGGL(k_transpose_gram, dim3(nblk), dim3(256), 0, st, W, D, H, Dp, (int)gt.x,
                       (int)gt.y, ngx, p.Pt32, hi, lo, z.A, p.G, z.B, p.hn_hi, p.hn_lo, p.pnorm);
  } else {
    hipLaunchKernelGGL(k_transpose, gt, dim3(256), 0, st, W, D, H, Dp, relu, p.Pt32, hi, lo, z.A,
                       z.B_dh ? z.B : nullptr);
    hipLaunchKernelGGL(k_norms, dim3((H + 3) / 4), dim3(256), 0, st, p.Pt32, Dp, H, p.hn_hi,
                       p.hn_lo, p.pnorm);
  }
  if (model == PROSPER_MCA)
    hipLaunchKernelGGL(k_rowmax, dim3((D + 255) / 256), dim3(256), 0, st, W, D, H, p.wmax);
  return hipGetLastError();
}

// Separate entry so that the theta kernel (which also clears pnorm) runs
// before the kernel that forms the norms (k_transpose_gram or k_norms) on the same stream.
hipError_t launch_theta_full(int model, int D, int H, double pi, double sigma,
                             const double* theta_dev, const Prepared& p, int32_t* redo_count,
                             hipStream_t st, int32_t* defer_count, float beta,
                             const DscParams& dsc, const AccZero& z) {
  hipLaunchKernelGGL(k_theta, dim3(1), dim3(64), 0, st, model, D, H, pi, sigma, theta_dev,
                     p.theta, p.pnorm, redo_count, defer_count, beta, dsc, z.scal, z.vcount,
                     z.nv);
  return hipGetLastError();
}

}  // namespace prosper
