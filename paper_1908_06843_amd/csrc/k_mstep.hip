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
//                in one wave's registers (lane i holds row i), then solves
//                64 of the rows below against it by forward substitution,
//                one thread per row, while another wave inverts the block.
//                The off-diagonal blocks of L are written to the lower
//                triangle and mirrored into the upper one, so that both
//                substitutions of the solve read coalesced rows; the
//                diagonal blocks are kept as their inverses (row-major and
//                transposed);
//   k_ms_syrk  : trailing update T -= P P^T on 32 x 32 tiles;
//   k_ms_solve : four pixels per workgroup: block forward and backward
//                substitution, each block step a few matrix-vector products
//                (the diagonal ones with the stored inverses) whose matrix
//                reads serve the four pixels; then W_new row d and its share
//                of tr(W_new^T A).
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
  double et_pi, et_s2;  // the selected-points variant's pi and sigma^2
};

// Workspace: header | M (H x H) | Dinv | DinvT (64 x 64 per diagonal block) |
// trp (D), each 256-byte aligned.
struct MstepWork {
  MstepHdr* hdr;
  double* M;
  double* Dinv;
  double* DinvT;
  double* trp;
};

static size_t dinv_bytes(int H) { return round_up((size_t)((H + NB - 1) / NB) * NB * NB * 8, 256); }

static MstepWork carve_mstep(void* work, int D, int H) {
  char* p = reinterpret_cast<char*>(work);
  MstepWork w;
  w.hdr = reinterpret_cast<MstepHdr*>(p);
  p += 256;
  w.M = reinterpret_cast<double*>(p);
  p += round_up((size_t)H * H * 8, 256);
  w.Dinv = reinterpret_cast<double*>(p);
  p += dinv_bytes(H);
  w.DinvT = reinterpret_cast<double*>(p);
  p += dinv_bytes(H);
  w.trp = reinterpret_cast<double*>(p);
  return w;
}

// M = symmetrised active block of B (+ jitter), identity on inactive latents.
// Every workgroup sums the active diagonal itself (H loads, in the same order
// everywhere, so all find the same jitter); workgroup 0 records the trace and
// clears the failure flag for the panels that follow.
__global__ __launch_bounds__(256) void k_ms_load(int H, const float* __restrict__ Bup,
                                                 MstepHdr* __restrict__ hdr,
                                                 double* __restrict__ M) {
  __shared__ double red[4];
  double t = 0.0;
  for (int h = threadIdx.x; h < H; h += 256) {
    const float b = Bup[(int64_t)h * H + h];
    if (b > 0.0f) t += (double)b;
  }
  t = wave_sum_d(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  const double trB = ((red[0] + red[1]) + red[2]) + red[3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->trB = trB;
    hdr->failed = 0;
  }
  const double jitter = 1e-12 * (trB > 0.0 ? trB / H : 1.0);
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
    // every read of the column is issued before the first update, so that
    // the reads overlap instead of each waiting out the LDS latency
    double cr[NBK];
    static_for<k + 1, NBK>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      cr[j] = col[j];
    });
    __builtin_amdgcn_sched_barrier(0);
    static_for<k + 1, NBK>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      a[j] = fma(-a[k], cr[j], a[j]);
    });
  });
  __builtin_amdgcn_sched_barrier(0);
}

// Forward substitution L_kk z = v for one vector per lane (v in z on entry),
// by columns: once z_m is final its multiples are taken off all later
// entries at once, so each step's chain is a single multiply and the updates
// within a step are independent of each other.  LT[m][c] = L_kk[c][m] (read
// by broadcast), inv[c] = 1 / L_kk[c][c].
__device__ __forceinline__ void subst_cols(double (&z)[NB], const double (*LT)[NB],
                                           const double* inv) {
  static_for<0, NB>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    // the step's reads first (they overlap), then its updates
    __builtin_amdgcn_sched_barrier(0);
    const double im = inv[m];
    double cr[NB];
    static_for<m + 1, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      cr[c] = LT[m][c];
    });
    __builtin_amdgcn_sched_barrier(0);
    z[m] *= im;
    static_for<m + 1, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      z[c] = fma(-cr[c], z[m], z[c]);
    });
  });
  __builtin_amdgcn_sched_barrier(0);
}

// Panel at kb (nb = min(64, H - kb) columns): factor the diagonal block
// L_kk in one wave's registers, then solve this workgroup's 64 rows below,
// L[i, kb:kb+nb] L_kk^T = M[i, kb:kb+nb], by forward substitution, one
// thread per row.  Every workgroup factors the (small) diagonal block
// itself.  Beside the rows below, wave 1 of workgroup 0 inverts L_kk
// (column j of L_kk^-1 by forward substitution of e_j, lane j; both
// substitutions by columns) and writes the inverse row-major (Dinv) and
// transposed (DinvT) for the solve: that is all that is kept of the diagonal
// block, whose place in M is left as it was (nothing reads it afterwards,
// and other workgroups may still be loading it).  Each row below is written
// to the lower triangle and mirrored into the upper one, so that both
// substitutions of the solve read coalesced rows.
__global__ __launch_bounds__(256) void k_ms_panel(int H, int kb, double* __restrict__ M,
                                                  double* __restrict__ Dinv,
                                                  double* __restrict__ DinvT,
                                                  MstepHdr* __restrict__ hdr) {
  __shared__ double LsT[NB][NB];  // LsT[m][c] = L_kk[c][m] (upper part zero)
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
      LsT[c][lane] = (c <= lane) ? a[c] : 0.0;
    });
    inv_s[lane] = myinv;
    if (blockIdx.x == 0 && bad && lane == 0) hdr->failed = 1;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid >= 64 && tid < 128) {
    const int64_t blk = (int64_t)(kb / NB) * NB * NB;
    double x[NB];
    static_for<0, NB>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      x[i] = i == lane ? 1.0 : 0.0;
    });
    subst_cols(x, LsT, inv_s);
    static_for<0, NB>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      Dinv[blk + i * NB + lane] = x[i];   // Dinv[i][lane] = L_kk^-1[i][lane]
      DinvT[blk + lane * NB + i] = x[i];  // DinvT[lane][i]
    });
    return;
  }
  // rows below the block exist only when the block is full (nb == 64); one
  // wave of them per workgroup (more waves sharing the broadcast reads of L
  // lengthened every row's chain)
  if (tid >= 64) return;
  const int i = kb + nb + blockIdx.x * 64 + tid;
  if (i >= H) return;
  double* xp = M + (int64_t)i * H + kb;
  double x[NB];
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    x[c] = xp[c];
  });
  // L_kk x = M[i, kb:kb+64]^T
  subst_cols(x, LsT, inv_s);
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

// x = B^-1 a_d for the SP pixels d = SP blockIdx.x + p, with the factor
// B = L L^T and the inverses of its 64 x 64 diagonal blocks:
//   forward   y_b = L_bb^-1 (a_b - sum_{k<b} L_bk y_k)
//   backward  x_b = L_bb^-T (y_b - sum_{k>b} L_kb^T x_k)
// Lane l owns row 64 b + l of each block step, for all SP pixels at once, so
// that every matrix element is loaded once per workgroup and serves the SP
// vectors (kept in LDS, read by broadcast).  The sum over the columns of a
// block step is split into quarters, one per wave; the partial sums are added
// in wave order and wave p finishes pixel p.  L_bk (k < b) is read from its
// mirror in the upper triangle and L_kb^T (k > b) from the lower one, so every
// matrix read of a wave is one coalesced 512-byte row; each wave's quarter of
// the diagonal block's inverse is loaded at the start of the step, with the
// off-diagonal rows.  Writes row d of W_new and its part of tr(W_new^T A).
constexpr int SP = 4;  // pixels per workgroup, one per wave

__global__ __launch_bounds__(256) void k_ms_solve(int D, int H, const float* __restrict__ A,
                                                  const float* __restrict__ Bup,
                                                  const double* __restrict__ M,
                                                  const double* __restrict__ Dinv,
                                                  const double* __restrict__ DinvT,
                                                  const MstepHdr* __restrict__ hdr,
                                                  const float* W_old, float* W_new,
                                                  double* __restrict__ trp) {
  extern __shared__ double sm_solve[];
  constexpr int Q = NB / 4;  // each wave's share of a diagonal block's columns
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Hpad = round_up(H, NB), nblk = Hpad / NB;
  double* xs = sm_solve;             // [SP][Hpad]   the vectors
  double* red = xs + SP * Hpad;      // [4][SP][64]  the waves' partial sums
  double* tb = red + 4 * SP * NB;    // [SP][64]     right-hand side of the diagonal step
  const int d0 = blockIdx.x * SP;
  const bool failed = hdr->failed != 0;
  for (int e = tid; e < SP * Hpad; e += 256) {
    const int p = e / Hpad, h = e - p * Hpad;
    const int d = min(d0 + p, D - 1);
    const int hc = h < H ? h : 0;
    const bool act = h < H && Bup[(int64_t)hc * H + hc] > 0.0f;
    const float a = A[(int64_t)d * H + hc];
    xs[e] = act ? (double)a : 0.0;
  }
  __syncthreads();
  // one block step: t = x_b - sum_j L(r, j) x_j over [j0, j1) split over the
  // waves, then x_b = Dg t with this wave's quarter dv of the diagonal factor
  auto step = [&](int b, int j0, int j1, const double* Dg) {
    const int r = NB * b + lane;
    const int rc = r < H ? r : H - 1;
    double dv[Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) dv[u] = Dg[(int64_t)(Q * wave + u) * NB + lane];
    double acc[SP];
#pragma unroll
    for (int p = 0; p < SP; ++p) acc[p] = 0.0;
    const int q = (j1 - j0 + 3) / 4;
    const int ja = j0 + wave * q, jb = min(ja + q, j1);
    // chunks of 16 rows whose loads are all issued before the first product
    // (addresses clamped into the range, values masked)
    for (int j = ja; j < jb; j += 16) {
      double mv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int jj = min(j + u, jb - 1);
        const double v = M[(int64_t)jj * H + rc];
        mv[u] = j + u < jb ? v : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int jj = min(j + u, jb - 1);
#pragma unroll
        for (int p = 0; p < SP; ++p) acc[p] = fma(-mv[u], xs[p * Hpad + jj], acc[p]);
      }
    }
#pragma unroll
    for (int p = 0; p < SP; ++p) red[(wave * SP + p) * NB + lane] = acc[p];
    __syncthreads();
    {
      double t = xs[wave * Hpad + r];
#pragma unroll
      for (int w = 0; w < 4; ++w) t += red[(w * SP + wave) * NB + lane];
      tb[wave * NB + lane] = r < H ? t : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < SP; ++p) acc[p] = 0.0;
#pragma unroll
    for (int u = 0; u < Q; ++u)
#pragma unroll
      for (int p = 0; p < SP; ++p) acc[p] = fma(dv[u], tb[p * NB + Q * wave + u], acc[p]);
#pragma unroll
    for (int p = 0; p < SP; ++p) red[(wave * SP + p) * NB + lane] = acc[p];
    __syncthreads();
    {
      double y = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) y += red[(w * SP + wave) * NB + lane];
      xs[wave * Hpad + r] = y;
    }
    __syncthreads();
  };
  // forward: rows of L_bk (k < b) from the mirror, M[j][r] = L[r][j];
  // DinvT[m][l] = L_bb^-1[l][m]
  for (int b = 0; b < nblk; ++b) step(b, 0, NB * b, DinvT + (int64_t)b * NB * NB);
  // backward: M[j][r] = L[j][r] for j beyond the block; Dinv[m][l] = L_bb^-1[m][l]
  for (int b = nblk - 1; b >= 0; --b) step(b, NB * (b + 1) < H ? NB * (b + 1) : H, H,
                                           Dinv + (int64_t)b * NB * NB);
  const int d = d0 + wave;
  if (d >= D) return;
  const int64_t row = (int64_t)d * H;
  const double* x = xs + wave * Hpad;
  if (failed) {
    for (int h = lane; h < H; h += 64) W_new[row + h] = W_old[row + h];
    if (lane == 0) trp[d] = 0.0;
    return;
  }
  double tr = 0.0;
  for (int h = lane; h < H; h += 64) {
    const bool act = Bup[(int64_t)h * H + h] > 0.0f;
    if (act) {
      tr = fma(x[h], (double)A[row + h], tr);
      W_new[row + h] = (float)x[h];
    } else {
      W_new[row + h] = W_old[row + h];
    }
  }
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

// DSC prior (the maximiser of sum_v vcount_v log pv_v on the simplex, with
// N H latents in all): pv_v = vcount_v / (N H) for v >= 1, pv_0 the rest.
__global__ void k_mstep_dsc_prior(int H, int nv, const double* __restrict__ scal,
                                  const double* __restrict__ vcount,
                                  double* __restrict__ theta_new) {
  if (threadIdx.x || blockIdx.x) return;
  const double NH = scal[4] * (double)H;
  double rest = 1.0;
  for (int v = 1; v < nv; ++v) {
    const double pv = vcount[v] / NH;
    theta_new[2 + v] = pv;
    rest -= pv;
  }
  theta_new[2] = rest;
}

hipError_t launch_mstep_dsc_prior(int H, int nv, const double* scal, const double* vcount,
                                  double* theta_new, hipStream_t st) {
  hipLaunchKernelGGL(k_mstep_dsc_prior, dim3(1), dim3(64), 0, st, H, nv, scal, vcount,
                     theta_new);
  return hipGetLastError();
}

// Selected-points M-step (prosper_mstep_et): one workgroup of 1024 threads.
// N_cut and the truncated-prior moments A, B from the E-step's pi; the
// N_cut-th largest logL by a radix select over order-preserving keys (four
// 8-bit digits, most significant first, a 256-bin histogram in LDS each);
// then the kept points' <k> and res summed in FP64, the points at the
// threshold key taken in index order when not all of them are kept.
__global__ __launch_bounds__(1024) void k_et_select(int64_t N, int D, int H, int gamma,
                                                    double pi_h,
                                                    const double* __restrict__ theta_dev,
                                                    const float* __restrict__ logL,
                                                    const float* __restrict__ k_mean,
                                                    const float* __restrict__ res,
                                                    MstepHdr* __restrict__ hdr) {
  __shared__ unsigned int hist[256];
  __shared__ uint32_t s_prefix;
  __shared__ int64_t s_need, s_cnt_eq;
  __shared__ double red_k[16], red_r[16];
  __shared__ int wcount[16];
  __shared__ int64_t s_taken;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double pi = theta_dev ? theta_dev[0] : pi_h;
  // A = P(#non-zero <= gamma), B = E[#non-zero; #non-zero <= gamma]
  double A = 0.0, B = 0.0;
  {
    double t = exp((double)H * log1p(-pi));  // k = 0
    for (int k = 0; k <= gamma && k <= H; ++k) {
      A += t;
      B += k * t;
      t *= (double)(H - k) / (double)(k + 1) * (pi / (1.0 - pi));
    }
  }
  int64_t n_cut = llround((double)N * A);
  n_cut = n_cut < 1 ? 1 : (n_cut > N ? N : n_cut);
  if (tid == 0) {
    s_prefix = 0u;
    s_need = n_cut;
  }
  // radix select of the n_cut-th largest key
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = tid; b < 256; b += 1024) hist[b] = 0u;
    __syncthreads();
    const uint32_t prefix = s_prefix;
    const uint32_t hmask = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
    for (int64_t n = tid; n < N; n += 1024) {
      const uint32_t key = f2key(logL[n]);
      if ((key & hmask) == (prefix & hmask)) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int64_t need = s_need, above = 0;
      int b = 255;
      for (; b > 0; --b) {
        if (above + (int64_t)hist[b] >= need) break;
        above += hist[b];
      }
      s_need = need - above;
      s_prefix = prefix | ((uint32_t)b << shift);
      if (shift == 0) s_cnt_eq = hist[b];
    }
    __syncthreads();
  }
  const uint32_t T = s_prefix;
  const int64_t need = s_need, cnt_eq = s_cnt_eq;
  // sums over the keys above T, and over all keys at T when all are kept
  double sk = 0.0, sr = 0.0;
  for (int64_t n = tid; n < N; n += 1024) {
    const uint32_t key = f2key(logL[n]);
    if (key > T || (key == T && need == cnt_eq)) {
      sk += (double)k_mean[n];
      sr += (double)res[n];
    }
  }
  // otherwise the first `need` points at T in index order: chunks of 1024
  // consecutive points, a block-wide prefix count of the points at T
  if (need < cnt_eq) {
    if (tid == 0) s_taken = 0;
    __syncthreads();
    for (int64_t base = 0; base < N; base += 1024) {
      const int64_t n = base + tid;
      const bool eq = n < N && f2key(logL[n]) == T;
      const uint64_t bal = ballot64(eq);
      if (lane == 0) wcount[wave] = __popcll(bal);
      __syncthreads();
      int64_t before = s_taken;
      for (int w = 0; w < wave; ++w) before += wcount[w];
      before += __popcll(bal & ((1ull << lane) - 1ull));
      if (eq && before < need) {
        sk += (double)k_mean[n];
        sr += (double)res[n];
      }
      __syncthreads();
      if (tid == 0) {
        int64_t t = s_taken;
        for (int w = 0; w < 16; ++w) t += wcount[w];
        s_taken = t;
      }
      __syncthreads();
    }
  }
  sk = wave_sum_d(sk);
  sr = wave_sum_d(sr);
  if (lane == 0) {
    red_k[wave] = sk;
    red_r[wave] = sr;
  }
  __syncthreads();
  if (tid == 0) {
    double tk = 0.0, tr = 0.0;
    for (int w = 0; w < 16; ++w) {
      tk += red_k[w];
      tr += red_r[w];
    }
    const double kbar = tk / (double)n_cut;
    hdr->et_pi = B > 0.0 ? pi * kbar * A / B : pi;
    hdr->et_s2 = tr / ((double)n_cut * (double)D);
  }
}

__global__ void k_et_finish(const MstepHdr* __restrict__ hdr, double* __restrict__ theta_new) {
  if (threadIdx.x || blockIdx.x) return;
  theta_new[0] = hdr->et_pi;
  theta_new[1] = sqrt(fmax(hdr->et_s2, 0.0));
}

hipError_t launch_mstep_et_select(int64_t N, int D, int H, int gamma, double pi,
                                  const double* theta_dev, const float* logL,
                                  const float* k_mean, const float* res, void* work,
                                  hipStream_t st) {
  const MstepWork w = carve_mstep(work, D, H);
  hipLaunchKernelGGL(k_et_select, dim3(1), dim3(1024), 0, st, N, D, H, gamma, pi, theta_dev, logL,
                     k_mean, res, w.hdr);
  return hipGetLastError();
}

hipError_t launch_mstep_et_finish(int D, int H, void* work, double* theta_new, hipStream_t st) {
  const MstepWork w = carve_mstep(work, D, H);
  hipLaunchKernelGGL(k_et_finish, dim3(1), dim3(64), 0, st, w.hdr, theta_new);
  return hipGetLastError();
}

size_t mstep_workspace_bytes(int model, int D, int H) {
  if (is_max_model(model)) return 256;
  return 256 + round_up((size_t)H * H * 8, 256) + 2 * dinv_bytes(H) + round_up((size_t)D * 8, 256);
}

hipError_t launch_mstep_factor(int model, int D, int H, const float* B, void* work,
                               hipStream_t st) {
  if (is_max_model(model)) return hipSuccess;
  if (H > 16 * 64) return hipErrorInvalidValue;
  const MstepWork w = carve_mstep(work, D, H);
  const int64_t HH = (int64_t)H * H;
  // at most 32 workgroups: when B is factored beside the A statistics only
  // the CUs those leave out are free, and more workgroups than fit there
  // wait for the statistics to end
  int64_t lb = (HH + 2047) / 2048;
  if (lb > 32) lb = 32;
  hipLaunchKernelGGL(k_ms_load, dim3((unsigned)lb), dim3(256), 0, st, H, B, w.hdr, w.M);
  for (int kb = 0; kb < H; kb += NB) {
    const int nb = (H - kb < NB) ? H - kb : NB;
    const int below = H - kb - nb;
    const unsigned nblk = below > 0 ? (unsigned)((below + 63) / 64) : 1u;
    hipLaunchKernelGGL(k_ms_panel, dim3(nblk), dim3(256), 0, st, H, kb, w.M, w.Dinv, w.DinvT,
                       w.hdr);
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
  const size_t lds = ((size_t)SP * round_up(H, NB) + 5 * SP * NB) * 8;
  hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(k_ms_solve), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ms_solve, dim3((unsigned)((D + SP - 1) / SP)), dim3(256), lds, st, D, H, A, B,
                     w.M, w.Dinv, w.DinvT, w.hdr, W_old, W_new, w.trp);
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
