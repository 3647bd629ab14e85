// Sufficient statistic A += y_n <s>_n^T on the candidate columns (row a8).
//
// Each workgroup owns a slice of DS pixels and a contiguous range of points
// and keeps a private H x DS partial of A in LDS; every point adds
// y_n[d] <s_j>_n into column sel_n[j] of the partial (LDS float atomics, so
// the four waves may update the same column).  The partial is flushed into
// A with one global atomic per non-zero entry.  Y is read once overall.
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

__global__ __launch_bounds__(256) void k_accum_A(const float* __restrict__ Y, int64_t N, int D,
                                                 int H, int Hp, const int32_t* __restrict__ sel,
                                                 const float* __restrict__ s_mean,
                                                 float* __restrict__ A, int DS, int nslices,
                                                 int64_t pts_per_group) {
  extern __shared__ float Ap[];  // [H][DS + 1]
  const int slice = blockIdx.x % nslices;
  const int64_t group = blockIdx.x / nslices;
  const int d0 = slice * DS;
  const int dlen = min(DS, D - d0);
  const int ld = DS + 1;
  for (int e = threadIdx.x; e < H * ld; e += 256) Ap[e] = 0.0f;
  __syncthreads();
  const int64_t nb = group * pts_per_group;
  const int64_t ne = min(N, nb + pts_per_group);
  if (nb < ne) {
    const int per = Hp * dlen;
    const int64_t total = (ne - nb) * per;
    for (int64_t e = threadIdx.x; e < total; e += 256) {
      const int64_t n = nb + e / per;
      const int rem = (int)(e % per);
      const int j = rem / dlen, d = rem % dlen;
      const int h = sel[n * Hp + j];
      atomicAdd(&Ap[h * ld + d], Y[n * D + d0 + d] * s_mean[n * Hp + j]);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < H * dlen; e += 256) {
    const int h = e % H, d = e / H;
    const float v = Ap[h * ld + d];
    if (v != 0.0f) atomicAdd(&A[(int64_t)(d0 + d) * H + h], v);
  }
}

hipError_t launch_accum_A(const float* Y, int64_t N, int D, int H, int Hp, const Scratch& s,
                          float* A, int num_cu, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  int DS = 128;
  while (DS > 1 && (size_t)H * (DS + 1) * 4 > 80 * 1024) DS /= 2;
  if (DS > D) DS = D;
  const int nslices = (D + DS - 1) / DS;
  int64_t ngroups = (2 * (int64_t)num_cu + nslices - 1) / nslices;
  if (ngroups < 1) ngroups = 1;
  if (ngroups > N) ngroups = N;
  const int64_t ppg = (N + ngroups - 1) / ngroups;
  ngroups = (N + ppg - 1) / ppg;
  const size_t lds = (size_t)H * (DS + 1) * 4;
  static size_t configured = 0;
  if (lds > configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_accum_A),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  hipLaunchKernelGGL(k_accum_A, dim3((unsigned)(ngroups * nslices)), dim3(256), lds, st, Y, N, D,
                     H, Hp, s.sel, s.s_mean, A, DS, nslices, ppg);
  return hipGetLastError();
}

}  // namespace prosper
