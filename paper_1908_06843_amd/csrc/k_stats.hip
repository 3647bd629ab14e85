// M-step sufficient statistics for linear superposition (row a8):
//   A (D x H) += sum_n y_n <s>_n^T       (columns sel_n only)
//   B (H x H, upper triangle) += sum_n <s s^T>_n   (block sel_n x sel_n only)
//
// Global float atomics are slow here (every workgroup of every XCD would hit
// the same few hundred KB), so the sums are formed without them: points are
// split into groups; per group one kind of workgroup keeps a D-slice x H
// partial of A in LDS and another a row block of B's packed upper triangle.
// Inside a workgroup the adds are LDS atomics; each workgroup then stores its
// partial with plain stores, and k_stats_reduce adds the group partials into
// A and B.  Y is read once overall.
//
// Per-point inputs (written by the state walk): sel (N x H'), <s> (N x H')
// and <s_i s_j> in pair-major layout ss[p][n], p < H' the diagonal
// <s_j^2>, then the pairs i < j in row-major order.
#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

static constexpr int BSLICE_MAX = 36 * 1024;  // floats of one B row block (144 KB)

// Row block b of B's upper triangle: rows [r0, r1) whose packed rows fit in
// BSLICE_MAX floats (greedy from row 0).
__host__ __device__ inline void bslice_bounds(int H, int b, int* r0, int* r1) {
  int start = 0, used = 0, cur = 0;
  for (int h = 0; h < H; ++h) {
    const int len = H - h;
    if (used + len > BSLICE_MAX) {
      if (cur == b) {
        *r0 = start;
        *r1 = h;
        return;
      }
      ++cur;
      start = h;
      used = 0;
    }
    used += len;
  }
  *r0 = (cur == b) ? start : H;
  *r1 = H;
}

__host__ __device__ inline int bslice_count(int H) {
  int n = 1, used = 0;
  for (int h = 0; h < H; ++h) {
    const int len = H - h;
    if (used + len > BSLICE_MAX) {
      ++n;
      used = 0;
    }
    used += len;
  }
  return n;
}

// packed offset of row h inside the block starting at r0
__host__ __device__ inline int bslice_off(int H, int r0, int h) {
  return (h - r0) * H - (h * (h - 1) - r0 * (r0 - 1)) / 2;
}

// A partials: workgroup = (point group, pixel slice [d0, d0 + dlen), dlen <= 64).
// Each wave takes tiles of 64 points: lane l first loads point l's candidate
// indices and <s>, and lane d the 64 pixels y[.][d0 + d]; then for every
// point p and candidate j the pair (sel, <s>) is broadcast with readlane and
// lane d adds y_p[d] <s_j> into column sel_j of the LDS partial.
template <int HPMAX>
__global__ __launch_bounds__(256) void k_stats_A(const float* __restrict__ Y, int64_t N, int D,
                                                 int H, int Hp, const int32_t* __restrict__ sel,
                                                 const float* __restrict__ s_mean, int DS, int nA,
                                                 int64_t pts_per_group, float* __restrict__ partA) {
  extern __shared__ float Ap[];  // [H][DS + 1]
  const int64_t group = blockIdx.x / nA;
  const int slice = blockIdx.x % nA;
  const int64_t nb = group * pts_per_group;
  const int64_t ne = min(N, nb + pts_per_group);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int d0 = slice * DS, dlen = min(DS, D - d0), ld = DS + 1;
  for (int e = threadIdx.x; e < H * ld; e += 256) Ap[e] = 0.0f;
  __syncthreads();
  for (int64_t t0 = nb + 64 * wave; t0 < ne; t0 += 256) {
    const int np = (int)min((int64_t)64, ne - t0);
    int sr[HPMAX];
    float mr[HPMAX];
#pragma unroll
    for (int j = 0; j < HPMAX; ++j) {
      const bool ok = j < Hp && lane < np;
      sr[j] = ok ? sel[(t0 + lane) * Hp + j] : 0;
      mr[j] = ok ? s_mean[(t0 + lane) * Hp + j] : 0.0f;
    }
    float yv[64];
#pragma unroll
    for (int p = 0; p < 64; ++p)
      yv[p] = (p < np && lane < dlen) ? Y[(t0 + p) * D + d0 + lane] : 0.0f;
#pragma unroll
    for (int p = 0; p < 64; ++p) {
#pragma unroll
      for (int j = 0; j < HPMAX; ++j) {
        if (j < Hp && p < np) {
          const int h = __builtin_amdgcn_readlane(sr[j], p);
          const float sv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mr[j]), p));
          if (lane < dlen) atomicAdd(&Ap[h * ld + lane], yv[p] * sv);
        }
      }
    }
  }
  __syncthreads();
  float* out = partA + ((int64_t)group * nA + slice) * ((int64_t)H * DS);
  for (int e = threadIdx.x; e < H * DS; e += 256) {
    const int h = e / DS, d = e % DS;
    out[e] = (d < dlen) ? Ap[h * ld + d] : 0.0f;
  }
}

// A partials on MFMA (D, H <= 256): A = Y^T S over tiles of 64 points, with
// S the points x H matrix holding <s_j> at column sel_j (at most H' non-zeros
// per row).  The S tile is scattered into LDS from (sel, <s>) and undone
// after use; both operands are split into BF16 head + tail and three
// products are summed (head*head + head*tail + tail*head) with FP32
// accumulation, which keeps the relative product error below 2^-16.
// Persistent workgroups (one wave per SIMD) keep their whole D x H partial
// in accumulator registers (wave w: row tiles w, w+4, w+8, w+12 x 16 column
// tiles) and store it once at the end.  Y rows are read whole (one 1 KB
// row per wave load) into an FP32 row-major tile; the transpose the MFMA
// needs (eight consecutive points of one pixel per lane) happens on the LDS
// reads.  The next tile's Y, sel and <s> are loaded into registers while the
// current tile is multiplied.
//   A operand (16 x 32): Y^T[d][pt], lane l: d = 16 rt + l % 16, points 8 (l / 16) .. + 8
//   B operand (32 x 16): S^T[h][pt],  lane l: h = 16 ct + l % 16, same points
static constexpr int AT_PTS = 64;         // points per tile (two k-steps of 32)
static constexpr int AT_LD = AT_PTS + 8;  // bf16 row stride of the transposed S tile
static constexpr int AT_YS = 258;         // float row stride of the Y tile

// FULL: D = H = 256, every row and column tile present (no per-MFMA tests).
template <int SELN, bool FULL>  // (sel, <s>) entries per thread and tile: 64 H' <= 256 SELN
__global__ __launch_bounds__(256, 1) void k_stats_A_mfma(
    const float* __restrict__ Y, int64_t N, int D, int H, int Hp, const int32_t* __restrict__ sel,
    const float* __restrict__ s_mean, float* __restrict__ partA) {
  __shared__ __align__(16) float Yf[AT_PTS * AT_YS];
  __shared__ __align__(16) bf16 Sh[256 * AT_LD], Sl[256 * AT_LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int Dt = FULL ? 16 : (D + 15) / 16, Ht = FULL ? 16 : (H + 15) / 16;
  const int64_t ntiles = (N + AT_PTS - 1) / AT_PTS;
  for (int e = tid; e < 256 * AT_LD; e += 256) {
    Sh[e] = (bf16)0.0f;
    Sl[e] = (bf16)0.0f;
  }
  for (int e = tid; e < AT_PTS * AT_YS; e += 256) Yf[e] = 0.0f;
  // every wave's zero fill must land before any wave scatters its first tile
  __syncthreads();
  f32x4 acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // thread -> float4 column c4 = lane of rows wave + 4 j (j < 16)
  const bool vec = (D & 3) == 0;
  const int c4 = lane, dd = 4 * c4;
  float4 yv[16];
  int sv_h[SELN];
  float sv_m[SELN];
  auto fetch = [&](int64_t t) {
    const int64_t n0 = t * AT_PTS;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t n = n0 + wave + 4 * j;
      const bool nok = n < N;
      const float* yr = Y + (nok ? n : N - 1) * D;
      if (vec) {
        const float4 x = *reinterpret_cast<const float4*>(yr + (dd < D ? dd : 0));
        yv[j] = (nok && dd < D) ? x : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        float e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float x = yr[min(dd + k, D - 1)];
          e[k] = (nok && dd + k < D) ? x : 0.f;
        }
        yv[j] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
    const int64_t nent = min((int64_t)AT_PTS, N - n0) * Hp;
#pragma unroll
    for (int u = 0; u < SELN; ++u) {
      const int64_t e = tid + 256 * u;
      const int64_t ec = e < nent ? e : 0;
      const int h = sel[n0 * Hp + ec];
      const float m = s_mean[n0 * Hp + ec];
      sv_h[u] = e < nent ? h : -1;
      sv_m[u] = m;
    }
  };
  if ((int64_t)blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // LDS is free: the previous tile's products and undo are complete
    if (dd < D) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        float2* dst = reinterpret_cast<float2*>(&Yf[(wave + 4 * j) * AT_YS + dd]);
        dst[0] = make_float2(yv[j].x, yv[j].y);
        dst[1] = make_float2(yv[j].z, yv[j].w);
      }
    }
    int cur_h[SELN];
#pragma unroll
    for (int u = 0; u < SELN; ++u) {
      cur_h[u] = sv_h[u];
      if (cur_h[u] >= 0) {
        const int pt = (tid + 256 * u) / Hp;
        const float v = sv_m[u];
        const bf16 hh = (bf16)v;
        Sh[cur_h[u] * AT_LD + pt] = hh;
        Sl[cur_h[u] * AT_LD + pt] = (bf16)(v - (float)hh);
      }
    }
    __syncthreads();
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);
#pragma unroll
    for (int ks = 0; ks < AT_PTS / 32; ++ks) {
      // A fragments of the wave's four row tiles once per k-step (the
      // transpose happens here), then each B fragment is read once and
      // used by all four
      bf16x8 ah[4], al[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int rt = wave + 4 * a;
        const float* col = &Yf[(32 * ks + 8 * q) * AT_YS + 16 * (rt < Dt ? rt : 0) + r16];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float v = col[e * AT_YS];
          const bf16 hv = (bf16)v;
          ah[a][e] = hv;
          al[a][e] = (bf16)(v - (float)hv);
        }
      }
#pragma unroll
      for (int ct = 0; ct < 16; ++ct) {
        if (FULL || ct < Ht) {
          const int ob = (16 * ct + r16) * AT_LD + 32 * ks + 8 * q;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Sh[ob]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Sl[ob]);
          // three passes over the four row tiles: consecutive MFMAs write
          // different accumulators, so none waits for the previous result
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (FULL || wave + 4 * a < Dt)
              acc[a][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh, acc[a][ct], 0, 0, 0);
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (FULL || wave + 4 * a < Dt)
              acc[a][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl, acc[a][ct], 0, 0, 0);
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (FULL || wave + 4 * a < Dt)
              acc[a][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh, acc[a][ct], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    // undo the scatter so the S tile is zero again
#pragma unroll
    for (int u = 0; u < SELN; ++u) {
      if (cur_h[u] >= 0) {
        const int pt = (tid + 256 * u) / Hp;
        Sh[cur_h[u] * AT_LD + pt] = (bf16)0.0f;
        Sl[cur_h[u] * AT_LD + pt] = (bf16)0.0f;
      }
    }
    __syncthreads();
  }
  float* out = partA + (int64_t)blockIdx.x * D * H;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int rt = wave + 4 * a;
    if (rt >= Dt) continue;
#pragma unroll
    for (int ct = 0; ct < 16; ++ct) {
      if (ct >= Ht) continue;
      const int h = 16 * ct + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int d = 16 * rt + 4 * q + i;
        if (d < D && h < H) out[(int64_t)d * H + h] = acc[a][ct][i];
      }
    }
  }
}

// A[d][h] += sum_g partA[g][d][h]; four consecutive entries per thread, eight
// partials in flight.
__global__ __launch_bounds__(256) void k_stats_A_reduce(int D, int H, int ng,
                                                        const float* __restrict__ partA,
                                                        float* __restrict__ A) {
  const int64_t n = (int64_t)D * H;
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e0 >= n) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = (n % 4 == 0);
  int g = 0;
  if (vec) {
    for (; g + 8 <= ng; g += 8) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = *reinterpret_cast<const float4*>(&partA[(int64_t)(g + u) * n + e0]);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[0] += v[u].x;
        acc[1] += v[u].y;
        acc[2] += v[u].z;
        acc[3] += v[u].w;
      }
    }
  }
  for (; g < ng; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (e0 + i < n) acc[i] += partA[(int64_t)g * n + e0 + i];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (e0 + i < n) A[e0 + i] += (float)acc[i];
}

// B partials from pair-major <s s^T> (kernels without their own B partial):
// workgroup = (point group, row block of B's packed upper triangle).
__global__ __launch_bounds__(256) void k_stats_B(int64_t N, int H, int Hp,
                                                 const int32_t* __restrict__ sel,
                                                 const float* __restrict__ ss, int nB,
                                                 int64_t pts_per_group, float* __restrict__ partB) {
  extern __shared__ float Bp[];
  const int64_t group = blockIdx.x / nB;
  const int b = blockIdx.x % nB;
  const int64_t nb = group * pts_per_group;
  const int64_t ne = min(N, nb + pts_per_group);
  int r0, r1;
  bslice_bounds(H, b, &r0, &r1);
  const int len = bslice_off(H, r0, r1);
  for (int e = threadIdx.x; e < len; e += 256) Bp[e] = 0.0f;
  __syncthreads();
  for (int64_t n = nb + threadIdx.x; n < ne; n += 256) {
    const int32_t* sn = sel + n * Hp;
    int p = Hp;
    for (int i = 0; i < Hp; ++i) {
      const int hi = sn[i];
      if (hi >= r0 && hi < r1) {
        const int base = bslice_off(H, r0, hi) - hi;
        atomicAdd(&Bp[base + hi], ss[(int64_t)i * N + n]);
        for (int j = i + 1; j < Hp; ++j)
          atomicAdd(&Bp[base + sn[j]], ss[(int64_t)(p + j - i - 1) * N + n]);
      }
      p += Hp - i - 1;
    }
  }
  __syncthreads();
  float* out = partB + ((int64_t)group * nB + b) * BSLICE_MAX;
  for (int e = threadIdx.x; e < len; e += 256) out[e] = Bp[e];
}

// A[d][h] += sum_g partA[g][d / DS][h][d % DS];  B[h][h2] += sum_g partB[g][slice(h)][...]
struct SliceRows {
  int r0[STATS_MAX_BSLICES + 1];
};

// B alone (A reduced by its own kernel): B[h][h2] += sum_g partB[g][slice(h)][...]
// for h2 >= h.  Threads run over the packed upper triangle (row h starts at
// h H - h (h - 1) / 2), four per element, each summing a quarter of the
// partials with 16 loads in flight; the four sums are added in quarter order.
__device__ __forceinline__ int64_t tri_row_start(int H, int h) {
  return (int64_t)h * H - (int64_t)h * (h - 1) / 2;
}

__global__ __launch_bounds__(256) void k_stats_reduce_B(int H, int nB, SliceRows rows, int ngB,
                                                        const float* __restrict__ partB,
                                                        float* __restrict__ B) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = e < (int64_t)H * (H + 1) / 2;
  double acc = 0.0;
  int h = 0, h2 = 0;
  if (ok) {
    // the row: the largest h with tri_row_start(h) <= e (root of the
    // quadratic, then corrected in integers)
    const double Hh = (double)H + 0.5;
    h = (int)(Hh - sqrt(Hh * Hh - 2.0 * (double)e));
    h = min(max(h, 0), H - 1);
    while (h > 0 && tri_row_start(H, h) > e) --h;
    while (h + 1 < H && tri_row_start(H, h + 1) <= e) ++h;
    h2 = h + (int)(e - tri_row_start(H, h));
    int b = 0;
    while (b + 1 < nB && h >= rows.r0[b + 1]) ++b;
    const int idx = bslice_off(H, rows.r0[b], h) + (h2 - h);
    const int per = (ngB + 3) / 4;
    const int g0 = q * per, g1 = min(g0 + per, ngB);
    int g = g0;
    for (; g + 16 <= g1; g += 16) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = partB[((int64_t)(g + u) * nB + b) * BSLICE_MAX + idx];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += v[u];
    }
    for (; g < g1; ++g) acc += partB[((int64_t)g * nB + b) * BSLICE_MAX + idx];
  }
  red[q][lane] = acc;
  __syncthreads();
  if (q == 0 && ok)
    B[(int64_t)h * H + h2] +=
        (float)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

__global__ __launch_bounds__(256) void k_stats_reduce(int D, int H, int DS, int nA, int nB,
                                                      SliceRows rows, int ngA, int ngB,
                                                      const float* __restrict__ partA,
                                                      const float* __restrict__ partB,
                                                      float* __restrict__ A, float* __restrict__ B) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nAe = (int64_t)D * H;
  if (e < nAe) {
    if (!A) return;  // A was reduced by its own kernel
    const int d = (int)(e / H), h = (int)(e % H);
    const int sl = d / DS, dd = d % DS;
    double acc = 0.0;
    int g = 0;
    for (; g + 8 <= ngA; g += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = partA[((int64_t)(g + u) * nA + sl) * ((int64_t)H * DS) + (int64_t)h * DS + dd];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; g < ngA; ++g)
      acc += partA[((int64_t)g * nA + sl) * ((int64_t)H * DS) + (int64_t)h * DS + dd];
    A[e] += (float)acc;
    return;
  }
  const int64_t f = e - nAe;
  if (f >= (int64_t)H * H) return;
  const int h = (int)(f / H), h2 = (int)(f % H);
  if (h2 < h) return;
  int b = 0;
  while (b + 1 < nB && h >= rows.r0[b + 1]) ++b;
  const int idx = bslice_off(H, rows.r0[b], h) + (h2 - h);
  double acc = 0.0;
  int g = 0;
  for (; g + 8 <= ngB; g += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partB[((int64_t)(g + u) * nB + b) * BSLICE_MAX + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; g < ngB; ++g) acc += partB[((int64_t)g * nB + b) * BSLICE_MAX + idx];
  B[f] += (float)acc;
}

StatsPlan stats_plan(int64_t N, int D, int H, int num_cu) {
  StatsPlan pl;
  int DS = 64;
  while (DS > 1 && (size_t)H * (DS + 1) * 4 > 80 * 1024) DS /= 2;
  if (DS > D) DS = D;
  pl.DS = DS;
  pl.nA = (D + DS - 1) / DS;
  pl.nB = bslice_count(H);
  int64_t ng = (2 * (int64_t)num_cu + pl.nA + pl.nB - 1) / (pl.nA + pl.nB);
  if (ng < 1) ng = 1;
  if (ng > N) ng = N > 0 ? N : 1;
  pl.ppg = (N + ng - 1) / ng;
  if (pl.ppg < 1) pl.ppg = 1;
  pl.ngroups = (int)((N + pl.ppg - 1) / pl.ppg);
  if (pl.ngroups < 1) pl.ngroups = 1;
  pl.partA_floats = (size_t)pl.ngroups * pl.nA * H * DS;
  pl.mfma_wgs = num_cu;
  if (stats_a_mfma_ok(D, H)) {
    const size_t m = (size_t)pl.mfma_wgs * D * H;
    if (m > pl.partA_floats) pl.partA_floats = m;
  }
  pl.partB_floats = (size_t)pl.ngroups * pl.nB * BSLICE_MAX;
  return pl;
}

int stats_bslice_floats() { return BSLICE_MAX; }
bool stats_a_mfma_ok(int D, int H) { return D <= 256 && H <= 256; }
int stats_bslice_count(int H) { return bslice_count(H); }

// B partials: either ngB = tree_blocks single-slice partials written by the
// training state walk (ss == NULL), or formed here from pair-major ss.  On
// the MFMA path B is completed first and `after_B` runs before the A
// statistics; reserve_cu CUs are then left out of the persistent A grid so
// that work forked by the hook finds room.
hipError_t launch_stats(const float* Y, int64_t N, int D, int H, int Hp, const Scratch& s,
                        const StatsPlan& pl, int tree_blocks, float* A, float* B,
                        hipStream_t st, int part, int reserve_cu) {
  if (N <= 0) return hipSuccess;
  const size_t ldsA = (size_t)H * (pl.DS + 1) * 4;
  const bool mfmaA = stats_a_mfma_ok(D, H);
  auto reduce_B_and_A = [&](bool with_A) -> hipError_t {
    int ngB = tree_blocks, nB = 1;
    if (s.ss) {
      const size_t ldsB = (size_t)BSLICE_MAX * 4;
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(k_stats_B), ldsB);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_stats_B, dim3((unsigned)(pl.ngroups * pl.nB)), dim3(256), ldsB, st, N,
                         H, Hp, s.sel, s.ss, pl.nB, pl.ppg, s.partB);
      ngB = pl.ngroups;
      nB = pl.nB;
    }
    SliceRows rows;
    for (int b = 0; b <= STATS_MAX_BSLICES; ++b) rows.r0[b] = H;
    for (int b = 0; b < nB; ++b) {
      int r0, r1;
      bslice_bounds(H, b, &r0, &r1);
      rows.r0[b] = r0;
    }
    if (!with_A) {
      const int64_t np = (int64_t)H * (H + 1) / 2;
      hipLaunchKernelGGL(k_stats_reduce_B, dim3((unsigned)((np + 63) / 64)), dim3(256), 0, st, H,
                         nB, rows, ngB, s.partB, B);
      return hipGetLastError();
    }
    const int64_t tot = (int64_t)D * H + (int64_t)H * H;
    hipLaunchKernelGGL(k_stats_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, D,
                       H, pl.DS, pl.nA, nB, rows, pl.ngroups, ngB, s.partA, s.partB, A, B);
    return hipGetLastError();
  };
  if (mfmaA) {
    if (part != STATS_A) {
      hipError_t e = reduce_B_and_A(false);
      if (e != hipSuccess || part == STATS_B) return e;
    }
    const int64_t ntiles = (N + AT_PTS - 1) / AT_PTS;
    int cap = pl.mfma_wgs - reserve_cu;
    if (cap < 1) cap = 1;
    const int nwg = (int)(ntiles < cap ? ntiles : cap);
    const bool full = D == 256 && H == 256;
    if (Hp <= 16 && full)
      hipLaunchKernelGGL((k_stats_A_mfma<4, true>), dim3((unsigned)nwg), dim3(256), 0, st, Y, N, D,
                         H, Hp, s.sel, s.s_mean, s.partA);
    else if (Hp <= 16)
      hipLaunchKernelGGL((k_stats_A_mfma<4, false>), dim3((unsigned)nwg), dim3(256), 0, st, Y, N,
                         D, H, Hp, s.sel, s.s_mean, s.partA);
    else
      hipLaunchKernelGGL((k_stats_A_mfma<8, false>), dim3((unsigned)nwg), dim3(256), 0, st, Y, N,
                         D, H, Hp, s.sel, s.s_mean, s.partA);
    const int64_t n = (int64_t)D * H;
    hipLaunchKernelGGL(k_stats_A_reduce, dim3((unsigned)((n / 4 + 256) / 256)), dim3(256), 0, st,
                       D, H, nwg, s.partA, A);
    return hipGetLastError();
  }
  // without the MFMA form A is formed first and reduced with B: all of it in
  // the B part, nothing left for the A part
  if (part == STATS_A) return hipSuccess;
  const int which = Hp <= 16 ? 0 : 1;
  const void* kern = which == 0 ? reinterpret_cast<const void*>(k_stats_A<16>)
                                : reinterpret_cast<const void*>(k_stats_A<32>);
  {
    hipError_t e = ensure_dynamic_lds(kern, ldsA);
    if (e != hipSuccess) return e;
  }
  const dim3 g((unsigned)(pl.ngroups * pl.nA));
  if (which == 0)
    hipLaunchKernelGGL(k_stats_A<16>, g, dim3(256), ldsA, st, Y, N, D, H, Hp, s.sel, s.s_mean,
                       pl.DS, pl.nA, pl.ppg, s.partA);
  else
    hipLaunchKernelGGL(k_stats_A<32>, g, dim3(256), ldsA, st, Y, N, D, H, Hp, s.sel, s.s_mean,
                       pl.DS, pl.nA, pl.ppg, s.partA);
  return reduce_B_and_A(true);
}

}  // namespace prosper
