// Internal interfaces of libprosper: device constants, workspace layout and
// the host-side launchers of every kernel.  Not part of the public ABI.
#pragma once

#include <functional>

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "prosper.h"

namespace prosper {

typedef __bf16 bf16;

// Derived constants of (pi, sigma) for one E-step call, computed on the
// device (so pi and sigma may themselves live on the device, as written by
// the M-step).  Log-joints inside the state walk are kept relative to the
// all-zero state and in log2 units:
//   lj(s) - lj(0) = k(s) c1 + lam (2 s^T b - s^T G s)            (BSC, TSC)
//   lj(s) - lj(0) = k(s) c1 - lam (||y - f(s)||^2 - ||y||^2)      (MCA)
//   lj(0)         = c0 - lam ||y||^2
// with c1 = log(pi/(1-pi)) (BSC, MCA) or log(pi/(2(1-pi))) (TSC),
// lam = 1/(2 sigma^2) and c0 = H log(1-pi) - D/2 log(2 pi sigma^2)
// (Eq. 1 prior, Eq. 2 Gaussian noise).
// DSC (discrete values phi_v, prior pv_v): the singleton term of value v is
//   u_v = log2(pv_v/pv_0) + lam2 (2 phi_v b - phi_v^2 G_hh),
// the pair term of values v, v' is -2 lam2 phi_v phi_v' G_hh', and
// c0 = H log(pv_0) - D/2 log(2 pi sigma^2).
static constexpr int DSC_MAXV = PROSPER_MAX_VALUES;
struct Theta {
  double pi, sigma;
  double c0;     // natural log
  float lam;     // 1/(2 sigma^2)
  float lam2;    // lam * log2(e)
  float c1_2;    // c1 * log2(e)
  float ln2;     // log(2)
  float beta;    // posterior temperature (1 = none)
  // DSC only (nv = 0 for the other models)
  int nv;                  // V
  float phi[DSC_MAXV];     // phi_v
  float u2[DSC_MAXV];      // log2(pv_v / pv_0)
  float cs[DSC_MAXV];      // sigma^2 ln(pv_v / pv_0): constant of the selection score
  double csd[DSC_MAXV];    // the same in FP64 (band re-scoring)
  float phimax, csmax;     // max_v |phi_v|, max_v |cs_v| (v >= 1; selection error bound)
};

// The DSC value set and prior of an argument block (host values).
struct DscParams {
  int nv = 0;
  float phi[DSC_MAXV] = {};
  double pv[DSC_MAXV] = {};
};
inline DscParams dsc_params(const prosper_args* a) {
  DscParams d;
  if (a->model == PROSPER_DSC) {
    d.nv = a->nvalues;
    for (int v = 0; v < DSC_MAXV; ++v) {
      d.phi[v] = a->phi[v];
      d.pv[v] = a->pv[v];
    }
  }
  return d;
}

// The posterior temperature of an argument block (0 stands for 1).
inline float args_beta(const prosper_args* a) { return a->beta == 0.0f ? 1.0f : a->beta; }

// Per-(model, W) derived data, rebuilt by k_prep for every E-step call.
struct Prepared {
  float* Pt32;      // H x Dp   projection rows: W^T (BSC/TSC) or max(W,0)^T (MCA), zero pad
  bf16* Pt_hi;      // H x Dp   BF16 head of Pt32 (BF16 precision only)
  bf16* Pt_lo;      // H x Dp   BF16 tail: Pt32 - Pt_hi rounded to BF16
  float* G;         // H x H    W^T W (BSC/TSC), FP64-accumulated then rounded
  float* hn_hi;     // H        1/2 ||P_h||^2 as an FP32 head ...
  float* hn_lo;     // H        ... and tail (FP64-accumulated)
  float* pnorm;     // 1        max_h ||P_h||_2
  float* wmax;      // Dp       max_h W_dh of the unclamped W (MCA: the superposition of
                    //          the state with all H latents active)
  Theta* theta;     // 1
};

// A += y <s>^T and B += <s s^T> through per-group LDS partials (no global atomics).
static constexpr int STATS_MAX_BSLICES = 32;
struct StatsPlan {
  int DS = 64, nA = 1, nB = 1, ngroups = 1, mfma_wgs = 256;
  int64_t ppg = 1;
  size_t partA_floats = 0, partB_floats = 0;
};
StatsPlan stats_plan(int64_t N, int D, int H, int num_cu);

// Per-call intermediates (device).
struct Scratch {
  int32_t* sel;     // N x H'
  float* bc;        // N x H'   candidate projections b_{I_n(j)} (signed)
  float* yy;        // N        ||y_n||^2 (FP32)
  float* s_mean;    // N x H'
  float* ss;        // H'(H'+1)/2 x N  <s_i s_j> per point, pair-major (statistics only)
  int32_t* redo_list;   // N   points the unrolled walk hands to the exact kernel
  int32_t* redo_count;  // 1   (cleared by the parameter kernel of each call)
  // Points whose selection needs the exact path, handed by the projection
  // kernel to a second kernel: defer_cap entries of (Hpad + 8) floats each
  // (header: point index as int64, cH, cN, delta; then the raw b row).
  // defer_cap == 0 keeps every such point inside the projection workgroup.
  float* defer = nullptr;
  int defer_cap = 0;
  int32_t* defer_count = nullptr;  // 1 (cleared by the parameter kernel of each call)
  // MCA/MMCA statistics of the unrolled walk: max_parts workgroup sums of
  // A and B (transposed, latents that fit in LDS), then A and B transposed
  // for the other latents (rows of D rounded up to 16); reduced into the
  // caller's accumulators at the end of the walk
  float* max_acc = nullptr;
  int max_parts = 0;
  float* partA;         // statistics: per-group partials of A and B
  float* partB;
  StatsPlan plan;
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Row length of the transposed projection matrix and of the staged Y tiles:
// the projection kernel reads 64 consecutive depths of a row per step.
inline int padded_depth(int D) { return round_up(D, 64); }

// Bump allocator over one device allocation (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base + off);
    off += n * sizeof(T);
    return p;
  }
};

// Host-side helpers shared by the ABI and the serving runtime.
// nv: the DSC value count (ignored by the other models).
void build_table(int model, int Hp, int gamma, std::vector<uint32_t>& act,
                 std::vector<uint32_t>& sgn, int nv = 0);
prosper_status count_states(int32_t model, int32_t Hp, int32_t gamma, int64_t* out,
                            std::string* msg, int nv = 0);
size_t prep_bytes(int Dp, int H, int prec);
Prepared carve_prep(void* base, int Dp, int H, int prec);

// Launchers (each returns the first HIP error it sees).
// Accumulators the preparation kernels clear (PROSPER_FLAG_ZERO_ACC): A is
// D x H; B is H x H, or D x H for the max models (B_dh).
struct AccZero {
  float* A = nullptr;
  float* B = nullptr;
  bool B_dh = false;
  double* scal = nullptr;
  double* vcount = nullptr;
  int nv = 0;
};
hipError_t launch_theta_full(int model, int D, int H, double pi, double sigma,
                             const double* theta_dev, const Prepared& p, int32_t* redo_count,
                             hipStream_t st, int32_t* defer_count = nullptr, float beta = 1.0f,
                             const DscParams& dsc = DscParams(), const AccZero& z = AccZero());
hipError_t launch_prep(int model, int prec, const float* W, int D, int H, int Dp,
                       const Prepared& p, hipStream_t st, const AccZero& z = AccZero());
// Entries of the projection's deferral list for N points: enough for a
// quarter of them (0 where every point takes the exact path anyway).
int project_defer_capacity(int64_t N, int H, int Hp, int prec = PROSPER_BF16);
hipError_t launch_project_select(int model, int prec, const float* Y, int64_t N, int D, int Dp,
                                 int H, int Hp, const Prepared& p, const Scratch& s,
                                 uint8_t* flagged, double* scal, hipStream_t st);
// BSC / TSC state walk.  tab_act/tab_sgn: canonical state table on the device.
// Statistics mode of the linear state walk (acc != NULL): either the
// training tree kernel writes per-workgroup B partials (returns the number
// of partials in *tree_blocks), or the walk writes pair-major <s s^T> into
// s.ss for the statistics kernel (*tree_blocks = 0).  Points handed to the
// exact kernel add their <s s^T> straight into acc_B with atomics.
// beta != 1 (annealing) and the per-point outputs k_out (<k>) and res_out
// (<||y - W s||^2>) always take the table-driven kernel.
hipError_t launch_states_lin(int model, int Hp, int gamma, int64_t N, int H, int64_t nstates,
                             const uint32_t* tab_act, const uint32_t* tab_sgn,
                             const Prepared& p, const Scratch& s, float* logL,
                             uint32_t* top_mask, float* top_q, int topk, bool acc,
                             float* acc_B, double* scal, int num_cu, int* tree_blocks,
                             hipStream_t st, float beta = 1.0f, float* k_out = nullptr,
                             float* res_out = nullptr);
// Max-superposition models: MCA and MMCA share the walk, statistics and M-step.
inline bool is_max_model(int m) { return m == PROSPER_MCA || m == PROSPER_MMCA; }
// DSC state walk (tab_code: 3-bit value codes of the actives): compiled for
// (H', gamma) = (8, 3) without top-k or annealing, else table-driven.  With
// acc, writes pair-major <s s^T> into s.ss for the statistics kernel and adds
// the expected value counts into vcount.
// Training (acc, compiled walk, B's packed triangle within a statistics
// slice): the walk writes per-workgroup B partials into s.partB instead
// (*tree_blocks = their number) and the redo points add into acc_B.
bool has_dsc_tree(int Hp, int gamma);
hipError_t launch_states_dsc(int Hp, int gamma, int64_t N, int H, int64_t nstates,
                             const uint32_t* tab_act, const uint32_t* tab_code, const Prepared& p,
                             const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, bool acc, double* vcount, double* scal, hipStream_t st,
                             float beta, int num_cu, int* tree_blocks, float* acc_B);
// MCA/MMCA state walk (max / largest-magnitude superposition).
hipError_t launch_states_max(int model, int Hp, int gamma, int64_t N, int D, int Dp, int H, int64_t nstates,
                             const uint32_t* tab_act, const float* Y, const Prepared& p,
                             const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, float* A_num, float* B_den, double* scal,
                             hipStream_t st);
int stats_bslice_floats();
bool stats_a_mfma_ok(int D, int H);
int stats_bslice_count(int H);
// Called on the E-step stream once B holds every contribution of the call
// (before the A statistics are formed), to queue work that needs only B.
typedef std::function<hipError_t(hipStream_t)> StatsHook;
// The statistics in two parts: STATS_B completes B (and, where A is not
// formed on MFMA, A too); STATS_A forms A (MFMA form; nothing otherwise).
// STATS_ALL is both on one stream.  The A part may run on another stream
// once the B part has been issued (it reads only the walk's outputs and Y).
enum { STATS_ALL = 0, STATS_B = 1, STATS_A = 2 };
hipError_t launch_stats(const float* Y, int64_t N, int D, int H, int Hp, const Scratch& s,
                        const StatsPlan& pl, int tree_blocks, float* A, float* B, hipStream_t st,
                        int part, int reserve_cu);
// M-step.
size_t mstep_workspace_bytes(int model, int D, int H);
hipError_t launch_mstep(int model, int D, int H, const float* A, const float* B,
                        const double* scal, const float* W_old, float* W_new,
                        double* theta_new, void* work, hipStream_t st);
// Selected-points M-step: pi and sigma^2 of the kept points into the M-step
// workspace (before the M-step proper), then copied into theta_new after it.
hipError_t launch_mstep_et_select(int64_t N, int D, int H, int gamma, double pi,
                                  const double* theta_dev, const float* logL,
                                  const float* k_mean, const float* res, void* work,
                                  hipStream_t st);
hipError_t launch_mstep_et_finish(int D, int H, void* work, double* theta_new, hipStream_t st);
// DSC prior update after the linear M-step: theta_new[2 + v] = pv_v.
hipError_t launch_mstep_dsc_prior(int H, int nv, const double* scal, const double* vcount,
                                  double* theta_new, hipStream_t st);
// The two halves of launch_mstep for BSC/TSC/DSC: factorisation of B into the
// workspace, and the solve + parameter update that uses it.
hipError_t launch_mstep_factor(int model, int D, int H, const float* B, void* work,
                               hipStream_t st);
hipError_t launch_mstep_solve(int model, int D, int H, const float* A, const float* B,
                              const double* scal, const float* W_old, float* W_new,
                              double* theta_new, void* work, hipStream_t st);

// Projection/preselection + state walk + A accumulation (after k_prep).
hipError_t launch_estep_core(int model, int prec, const float* Y, int64_t N, int D, int H, int Hp,
                             int gamma, int64_t ns, const uint32_t* tab_act,
                             const uint32_t* tab_sgn, const Prepared& p, const Scratch& sc,
                             uint8_t* flagged, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, float* A, float* B, double* scal, int num_cu,
                             hipStream_t s);

// Raise a kernel's dynamic-LDS limit to at least `bytes` (once per kernel and
// size; safe to call from several host threads).
hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes);

// E-step launch sequence shared by the entry points (host.hip).
// Checks of an E-step call (validate_args plus pointer requirements).
prosper_status check_estep(const prosper_args* a, const float* Y, const float* W,
                           const prosper_point_out* out, const prosper_acc* acc,
                           std::string* msg, int64_t* ns);
// Per-point workspace of one E-step call: which pieces it needs and its size.
struct EstepLayout {
  bool need_sel = false, need_sm = false, lin_acc = false, tree_acc = false, max_acc = false;
  int defer_cap = 0, Hpad = 0, max_parts = 0;
  size_t npairs = 0, partB_floats = 0, bytes = 0;
  StatsPlan plan;
};
// num_cu sizes the statistics partials (one per walk / statistics
// workgroup); defer_cap is the length of the projection's deferral list.
EstepLayout plan_estep(const prosper_args* a, const prosper_point_out* out, int num_cu,
                       int defer_cap);
Scratch carve_estep(void* base, const EstepLayout& L, const prosper_args* a,
                    const prosper_point_out* out);
// Parameter prep, projection + preselection, state walk and statistics of one
// E-step on stream s.  c may be NULL (no profiling).  after_B runs once B is
// complete; reserve_cu CUs are left free for work it forks.
// num_cu: the CU count the statistics partials of the layout were planned for.
// With after_B and a_stream, the A statistics run on a_stream after the hook
// (which the caller uses to queue B's factorisation on s); the caller joins
// a_stream back into s.
hipError_t enqueue_estep(prosper_ctx* c, const prosper_args* a, const float* Y, const float* W,
                         const prosper_point_out* out, const prosper_acc* acc, hipStream_t s,
                         const Prepared& p, const Scratch& sc, const uint32_t* tab_act,
                         const uint32_t* tab_sgn, int64_t ns, int num_cu,
                         const StatsHook& after_B, int reserve_cu,
                         hipStream_t a_stream = nullptr);
// Records the text of a failure of a context-less call (prosper_last_error(NULL)).
prosper_status set_error(prosper_status st, const std::string& msg);

// Whether a compile-time specialised state walk exists for this shape.
bool has_tree_kernel(int model, int Hp, int gamma);
// The same for max superposition (also depends on D and H).
bool has_max_tree(int Hp, int gamma, int D, int H);
size_t max_tree_acc_floats(int D, int H, int nparts);
hipError_t launch_states_max_tree(int model, int Hp, int gamma, int64_t N, int D, int Dp, int H,
                                  const uint32_t* tab_act, const float* Y, const Prepared& p,
                                  const Scratch& s, float* logL, uint32_t* top_mask, float* top_q,
                                  int topk, float* A_num, float* B_den, double* scal,
                                  hipStream_t st);

}  // namespace prosper
