// Host side of libprosper: the C ABI of prosper.h -- argument validation,
// the canonical state table, the context (device workspace, cached state
// tables) and the launch sequence of one E-step / M-step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "prosper_internal.hpp"

namespace prosper {
size_t project_lds_bytes(int Dp, int H, int prec, int tm);
size_t states_max_lds_bytes(int Hp, int D, int64_t nstates, bool acc);
}  // namespace prosper

using namespace prosper;

namespace {

thread_local std::string g_tls_err;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Table {
  uint32_t* act = nullptr;
  uint32_t* sgn = nullptr;
  int64_t count = 0;
};

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

struct ProfEntry {
  double ms = 0.0;
  int64_t launches = 0;
};

struct prosper_ctx {
  int device = 0;
  int num_cu = 256;
  std::string err;
  DevBuf prep, scratch, mwork;
  std::map<std::tuple<int, int, int>, Table> tables;
  // per-kernel-group timing
  bool prof = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::tuple<const char*, hipEvent_t, hipEvent_t>> ev_pending;
  std::map<std::string, ProfEntry> prof_tab;
  std::vector<std::string> prof_order;
  std::string prof_only;  // time only this group ("" = every group)
  // B factored ahead by an E-step (PROSPER_FLAG_FACTOR_B) on the side stream
  hipStream_t side = nullptr;
  hipEvent_t ev_b = nullptr, ev_f = nullptr;
  bool factor_ready = false;
  const float* factor_B = nullptr;
  int factor_model = -1, factor_D = 0, factor_H = 0;
};

namespace {

prosper_status fail(prosper_ctx* c, prosper_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_tls_err = msg;
  return st;
}

prosper_status hip_fail(prosper_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return fail(c, PROSPER_EDEVICE, m);
}

// grow-only device buffer; freeing waits for the device (hipFree does)
hipError_t ensure(DevBuf& b, size_t bytes) {
  if (b.cap >= bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t cap = bytes + bytes / 4 + 4096;
  hipError_t e = hipMalloc(&b.p, cap);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.cap = cap;
  return hipSuccess;
}

}  // namespace

namespace prosper {
prosper_status set_error(prosper_status st, const std::string& msg) {
  g_tls_err = msg;
  return st;
}

hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  size_t& have = done[kernel];
  if (have >= bytes) return hipSuccess;
  hipError_t e =
      hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) have = bytes;
  return e;
}

// Canonical enumeration: k ascending, slot tuples lexicographic, TSC sign
// codes counting up (bit i of the code = sign of the i-th active slot), DSC
// value codes of one support counting up in base V-1 (digit i, plus one, is
// the value code of the i-th active slot, stored in bits 3i .. 3i+2).
void build_table(int model, int Hp, int gamma, std::vector<uint32_t>& act,
                 std::vector<uint32_t>& sgn, int nv) {
  act.clear();
  sgn.clear();
  const int kmax = gamma < Hp ? gamma : Hp;
  for (int k = 0; k <= kmax; ++k) {
    std::vector<int> c(k);
    for (int i = 0; i < k; ++i) c[i] = i;
    while (true) {
      uint32_t a = 0;
      for (int i = 0; i < k; ++i) a |= 1u << c[i];
      if (model == PROSPER_DSC) {
        int64_t ncodes = 1;
        for (int i = 0; i < k; ++i) ncodes *= nv - 1;
        for (int64_t code = 0; code < ncodes; ++code) {
          uint32_t w = 0;
          int64_t r = code;
          for (int i = 0; i < k; ++i) {
            w |= (uint32_t)(1 + r % (nv - 1)) << (3 * i);
            r /= nv - 1;
          }
          act.push_back(a);
          sgn.push_back(w);
        }
      } else if (model == PROSPER_TSC) {
        for (uint32_t code = 0; code < (1u << k); ++code) {
          uint32_t s = 0;
          for (int i = 0; i < k; ++i)
            if ((code >> i) & 1u) s |= 1u << c[i];
          act.push_back(a);
          sgn.push_back(s);
        }
      } else {
        act.push_back(a);
        sgn.push_back(0u);
      }
      // next combination in lexicographic order
      int i = k - 1;
      while (i >= 0 && c[i] == Hp - k + i) --i;
      if (i < 0) break;
      ++c[i];
      for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
    }
  }
}

prosper_status count_states(int32_t model, int32_t Hp, int32_t gamma, int64_t* out,
                            std::string* msg, int nv) {
  if (model != PROSPER_BSC && model != PROSPER_TSC && model != PROSPER_DSC &&
      !is_max_model(model)) {
    if (msg) *msg = "unknown model";
    return PROSPER_EINVAL;
  }
  if (model == PROSPER_DSC && (nv < 2 || nv > PROSPER_MAX_VALUES)) {
    if (msg) *msg = "DSC nvalues outside 2..8";
    return PROSPER_EINVAL;
  }
  if (Hp < 1 || Hp > PROSPER_MAX_HPRIME) {
    if (msg) *msg = "Hprime outside 1..32";
    return PROSPER_EINVAL;
  }
  if (gamma < 0 || gamma > Hp) {
    if (msg) *msg = "gamma outside 0..Hprime";
    return PROSPER_EINVAL;
  }
  if (model == PROSPER_DSC && gamma > PROSPER_DSC_MAX_GAMMA) {
    if (msg) *msg = "DSC gamma above 10 (3-bit value codes of the actives)";
    return PROSPER_EINVAL;
  }
  const int V1 = (model == PROSPER_TSC) ? 2 : (model == PROSPER_DSC ? nv - 1 : 1);
  double total = 0.0;
  int64_t cnt = 0, pw = 1;
  for (int k = 0; k <= gamma; ++k) {
    const double t = (double)binom(Hp, k) * std::pow((double)V1, k);
    total += t;
    if (total > (double)PROSPER_MAX_STATES) {
      if (msg) *msg = "truncated state set larger than PROSPER_MAX_STATES";
      return PROSPER_EINVAL;
    }
    cnt += binom(Hp, k) * pw;
    pw *= V1;
  }
  *out = cnt;
  return PROSPER_OK;
}
}  // namespace prosper

namespace {

prosper_status validate(const prosper_args* a, std::string* msg, int64_t* nstates) {
  if (!a) {
    *msg = "args is NULL";
    return PROSPER_EINVAL;
  }
  if (a->model != PROSPER_BSC && a->model != PROSPER_TSC && a->model != PROSPER_DSC &&
      !is_max_model(a->model)) {
    *msg = "unknown model";
    return PROSPER_EINVAL;
  }
  const bool dsc = a->model == PROSPER_DSC;
  if (dsc) {
    if (a->nvalues < 2 || a->nvalues > PROSPER_MAX_VALUES) {
      *msg = "DSC nvalues outside 2..8";
      return PROSPER_EINVAL;
    }
    if (a->phi[0] != 0.0f) {
      *msg = "DSC phi[0] must be 0";
      return PROSPER_EINVAL;
    }
    for (int v = 1; v < a->nvalues; ++v) {
      if (!std::isfinite(a->phi[v]) || a->phi[v] == 0.0f) {
        *msg = "DSC phi[1..V-1] must be finite and non-zero";
        return PROSPER_EINVAL;
      }
      for (int w = 1; w < v; ++w)
        if (a->phi[w] == a->phi[v]) {
          *msg = "DSC phi values must be distinct";
          return PROSPER_EINVAL;
        }
    }
    if (!a->theta_dev) {
      double sum = 0.0;
      for (int v = 0; v < a->nvalues; ++v) {
        if (!(a->pv[v] > 0.0) || !std::isfinite(a->pv[v])) {
          *msg = "DSC pv entries must be positive";
          return PROSPER_EINVAL;
        }
        sum += a->pv[v];
      }
      if (std::fabs(sum - 1.0) > 1e-9) {
        *msg = "DSC pv must sum to 1";
        return PROSPER_EINVAL;
      }
    }
  }
  if (a->precision != PROSPER_FP32 && a->precision != PROSPER_BF16 &&
      a->precision != PROSPER_BF16X1) {
    *msg = "unknown precision";
    return PROSPER_EINVAL;
  }
  if (a->N < 0) {
    *msg = "N < 0";
    return PROSPER_EINVAL;
  }
  if (a->D < 1 || a->D > PROSPER_MAX_D) {
    *msg = "D outside 1..1024";
    return PROSPER_EINVAL;
  }
  if (a->H < 1 || a->H > PROSPER_MAX_H) {
    *msg = "H outside 1..1024";
    return PROSPER_EINVAL;
  }
  if (a->Hprime < 1 || a->Hprime > a->H || a->Hprime > PROSPER_MAX_HPRIME) {
    *msg = "Hprime outside 1..min(H, 32)";
    return PROSPER_EINVAL;
  }
  if (a->gamma < 0 || a->gamma > a->Hprime) {
    *msg = "gamma outside 0..Hprime";
    return PROSPER_EINVAL;
  }
  if (!a->theta_dev) {
    if (!dsc && !(a->pi > 0.0 && a->pi < 1.0)) {
      *msg = "pi outside (0, 1)";
      return PROSPER_EINVAL;
    }
    if (!(a->sigma > 0.0) || !std::isfinite(a->sigma)) {
      *msg = "sigma must be positive and finite";
      return PROSPER_EINVAL;
    }
  }
  if (a->topk < 0 || a->topk > PROSPER_MAX_TOPK) {
    *msg = "topk outside 0..8";
    return PROSPER_EINVAL;
  }
  if (a->accumulate != 0 && a->accumulate != 1) {
    *msg = "accumulate must be 0 or 1";
    return PROSPER_EINVAL;
  }
  if (!(a->beta == 0.0f || (a->beta > 0.0f && a->beta <= 1.0f))) {
    *msg = "beta (posterior temperature) outside (0, 1]";
    return PROSPER_EINVAL;
  }
  if ((a->flags & ~(PROSPER_FLAG_FACTOR_B | PROSPER_FLAG_ZERO_ACC)) != 0u) {
    *msg = "unknown flag bits";
    return PROSPER_EINVAL;
  }
  if ((a->flags & PROSPER_FLAG_ZERO_ACC) && !a->accumulate) {
    *msg = "PROSPER_FLAG_ZERO_ACC needs accumulate = 1";
    return PROSPER_EINVAL;
  }
  if ((a->flags & PROSPER_FLAG_FACTOR_B) && (!a->accumulate || is_max_model(a->model))) {
    *msg = "PROSPER_FLAG_FACTOR_B needs accumulate = 1 and a linear model (BSC/TSC/DSC)";
    return PROSPER_EINVAL;
  }
  int64_t ns = 0;
  prosper_status st = count_states(a->model, a->Hprime, a->gamma, &ns, msg, a->nvalues);
  if (st != PROSPER_OK) return st;
  if (a->topk > ns) {
    *msg = "topk larger than the truncated state set";
    return PROSPER_EINVAL;
  }
  if (is_max_model(a->model)) {
    const size_t lds = states_max_lds_bytes(a->Hprime, a->D, ns, a->accumulate != 0);
    if (lds > 150 * 1024 && !has_max_tree(a->Hprime, a->gamma, a->D, a->H)) {
      *msg = "MCA shape (Hprime x D and |K|) exceeds the per-workgroup LDS of this build";
      return PROSPER_EINVAL;
    }
  }
  if (nstates) *nstates = ns;
  return PROSPER_OK;
}

prosper_status get_table(prosper_ctx* c, int model, int Hp, int gamma, Table** out,
                         int nv = 0) {
  // DSC tables differ by the value count
  const int kind = is_max_model(model) ? PROSPER_BSC : (model == PROSPER_DSC ? 100 + nv : model);
  auto key = std::make_tuple(kind, Hp, gamma);
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    *out = &it->second;
    return PROSPER_OK;
  }
  std::vector<uint32_t> act, sgn;
  build_table(model, Hp, gamma, act, sgn, nv);
  Table t;
  t.count = (int64_t)act.size();
  hipError_t e = hipMalloc(&t.act, act.size() * 4);
  if (e == hipSuccess) e = hipMalloc(&t.sgn, sgn.size() * 4);
  if (e == hipSuccess) e = hipMemcpy(t.act, act.data(), act.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(t.sgn, sgn.data(), sgn.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (t.act) hipFree(t.act);
    if (t.sgn) hipFree(t.sgn);
    return hip_fail(c, e, "state table upload");
  }
  auto ins = c->tables.emplace(key, t);
  *out = &ins.first->second;
  return PROSPER_OK;
}



}  // namespace

namespace prosper {
size_t prep_bytes(int Dp, int H, int prec) {
  size_t b = 0;
  auto add = [&](size_t n) { b = ((b + 255) & ~(size_t)255) + n; };
  add((size_t)H * Dp * 4);
  add(prec != PROSPER_FP32 ? (size_t)H * Dp * 2 : 0);
  add(prec != PROSPER_FP32 ? (size_t)H * Dp * 2 : 0);
  add((size_t)H * H * 4);
  add((size_t)H * 4);
  add((size_t)H * 4);
  add(4);
  add((size_t)Dp * 4);
  add(sizeof(Theta));
  return b + 256;
}

Prepared carve_prep(void* base, int Dp, int H, int prec) {
  Carve cv{reinterpret_cast<char*>(base)};
  Prepared p;
  p.Pt32 = cv.take<float>((size_t)H * Dp);
  p.Pt_hi = cv.take<bf16>(prec != PROSPER_FP32 ? (size_t)H * Dp : 0);
  p.Pt_lo = cv.take<bf16>(prec != PROSPER_FP32 ? (size_t)H * Dp : 0);
  p.G = cv.take<float>((size_t)H * H);
  p.hn_hi = cv.take<float>(H);
  p.hn_lo = cv.take<float>(H);
  p.pnorm = cv.take<float>(1);
  p.wmax = cv.take<float>(Dp);
  p.theta = cv.take<Theta>(1);
  return p;
}
}  // namespace prosper


namespace {
hipEvent_t prof_event(prosper_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// Runs `launch` between two events on stream s when profiling is enabled.
template <typename F>
hipError_t timed(prosper_ctx* c, const char* name, hipStream_t s, F&& launch) {
  if (!c || !c->prof || (!c->prof_only.empty() && c->prof_only != name)) return launch();
  hipEvent_t a = prof_event(c), b = prof_event(c);
  hipEventRecord(a, s);
  hipError_t e = launch();
  hipEventRecord(b, s);
  c->ev_pending.emplace_back(name, a, b);
  return e;
}

void prof_collect(prosper_ctx* c) {
  for (auto& t : c->ev_pending) {
    hipEvent_t a = std::get<1>(t), b = std::get<2>(t);
    hipEventSynchronize(b);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, a, b);
    std::string name = std::get<0>(t);
    if (!c->prof_tab.count(name)) c->prof_order.push_back(name);
    c->prof_tab[name].ms += ms;
    c->prof_tab[name].launches += 1;
    c->ev_free.push_back(a);
    c->ev_free.push_back(b);
  }
  c->ev_pending.clear();
}
}  // namespace

namespace prosper {
// Launch sequence of one E-step after the parameter preparation: projection
// and preselection, state walk, A accumulation.  Shared by prosper_estep and
// the serving runtime (which prepares its dictionary once).
hipError_t launch_estep_core(int model, int prec, const float* Y, int64_t N, int D, int H, int Hp,
                             int gamma, int64_t ns, const uint32_t* tab_act,
                             const uint32_t* tab_sgn, const Prepared& p, const Scratch& sc,
                             uint8_t* flagged, float* logL, uint32_t* top_mask, float* top_q,
                             int topk, float* A, float* B, double* scal, int num_cu,
                             hipStream_t s) {
  const int Dp = padded_depth(D);
  hipError_t e = launch_project_select(model, prec, Y, N, D, Dp, H, Hp, p, sc, flagged, scal, s);
  if (e != hipSuccess) return e;
  if (is_max_model(model))
    return launch_states_max(model, Hp, gamma, N, D, Dp, H, ns, tab_act, Y, p, sc, logL, top_mask, top_q,
                             topk, A, B, scal, s);
  int tree_blocks = 0;
  e = launch_states_lin(model, Hp, gamma, N, H, ns, tab_act, tab_sgn, p, sc, logL, top_mask,
                        top_q, topk, A != nullptr, B, scal, num_cu, &tree_blocks, s);
  if (e == hipSuccess && A)
    e = launch_stats(Y, N, D, H, Hp, sc, sc.plan, tree_blocks, A, B, s, STATS_ALL, 0);
  return e;
}
}  // namespace prosper

namespace prosper {

// Argument checks shared by the E-step entry points.
prosper_status check_estep(const prosper_args* a, const float* Y, const float* W,
                           const prosper_point_out* out, const prosper_acc* acc,
                           std::string* msg, int64_t* ns) {
  prosper_status st = validate(a, msg, ns);
  if (st != PROSPER_OK) return st;
  if (a->N == 0) return PROSPER_OK;
  if (!Y || !W) {
    *msg = "Y or W is NULL";
    return PROSPER_EINVAL;
  }
  if (a->accumulate && (!acc || !acc->A || !acc->B || !acc->scal)) {
    *msg = "accumulate=1 needs acc->A, acc->B and acc->scal";
    return PROSPER_EINVAL;
  }
  if (out && (out->k_mean || out->res) && a->model != PROSPER_BSC &&
      a->model != PROSPER_TSC) {
    *msg = "k_mean and res outputs are defined for BSC and TSC";
    return PROSPER_EINVAL;
  }
  if (a->accumulate && a->model == PROSPER_DSC && !acc->vcount) {
    *msg = "DSC with accumulate=1 needs acc->vcount";
    return PROSPER_EINVAL;
  }
  if (a->topk > 0 && out && !out->top_mask && !out->top_q) {
    *msg = "topk > 0 needs top_mask or top_q";
    return PROSPER_EINVAL;
  }
  return PROSPER_OK;
}

// num_cu sizes the statistics partials (one per walk / statistics
// workgroup); defer_cap is the length of the projection's deferral list.
EstepLayout plan_estep(const prosper_args* a, const prosper_point_out* out, int num_cu,
                       int defer_cap) {
  EstepLayout L;
  const int64_t N = a->N;
  const int D = a->D, H = a->H, Hp = a->Hprime;
  L.need_sel = !(out && out->sel);
  L.need_sm = !(out && out->s_mean);
  L.Hpad = (H + 63) / 64 * 64;
  L.defer_cap = defer_cap;
  L.lin_acc = a->accumulate && !is_max_model(a->model);
  L.npairs = (size_t)Hp * (Hp + 1) / 2;
  L.plan = stats_plan(N, D, H, num_cu);
  L.tree_acc = L.lin_acc && a->topk == 0 && args_beta(a) == 1.0f &&
               !(out && (out->k_mean || out->res)) &&
               (has_tree_kernel(a->model, Hp, a->gamma) ||
                (a->model == PROSPER_DSC && has_dsc_tree(Hp, a->gamma))) &&
               (int64_t)H * (H + 1) / 2 <= stats_bslice_floats();
  L.partB_floats = L.tree_acc ? (size_t)num_cu * stats_bslice_floats() : L.plan.partB_floats;
  L.max_acc = a->accumulate && is_max_model(a->model) && has_max_tree(Hp, a->gamma, D, H);
  L.max_parts = num_cu;
  size_t sb = 0;
  auto add = [&](size_t n) { sb = ((sb + 255) & ~(size_t)255) + n; };
  add(L.need_sel ? (size_t)N * Hp * 4 : 0);
  add((size_t)N * Hp * 4);
  add((size_t)N * 4);
  add(L.need_sm ? (size_t)N * Hp * 4 : 0);
  add((size_t)N * 4);
  add(8);
  add((size_t)defer_cap * (L.Hpad + 8) * 4);
  add(L.lin_acc && !L.tree_acc ? L.npairs * N * 4 : 0);
  add(L.lin_acc ? L.plan.partA_floats * 4 : 0);
  add(L.lin_acc ? L.partB_floats * 4 : 0);
  add(L.max_acc ? max_tree_acc_floats(D, H, L.max_parts) * 4 : 0);
  L.bytes = sb;
  return L;
}

Scratch carve_estep(void* base, const EstepLayout& L, const prosper_args* a,
                    const prosper_point_out* out) {
  const int64_t N = a->N;
  const int Hp = a->Hprime;
  Carve cv{reinterpret_cast<char*>(base)};
  Scratch sc;
  int32_t* sel_ws = cv.take<int32_t>(L.need_sel ? (size_t)N * Hp : 0);
  sc.bc = cv.take<float>((size_t)N * Hp);
  sc.yy = cv.take<float>((size_t)N);
  float* sm_ws = cv.take<float>(L.need_sm ? (size_t)N * Hp : 0);
  sc.redo_list = cv.take<int32_t>((size_t)N);
  sc.redo_count = cv.take<int32_t>(2);
  sc.defer_count = sc.redo_count + 1;
  sc.defer = cv.take<float>((size_t)L.defer_cap * (L.Hpad + 8));
  sc.defer_cap = L.defer_cap;
  sc.ss = cv.take<float>(L.lin_acc && !L.tree_acc ? L.npairs * N : 0);
  if (!(L.lin_acc && !L.tree_acc)) sc.ss = nullptr;
  sc.partA = cv.take<float>(L.lin_acc ? L.plan.partA_floats : 0);
  sc.partB = cv.take<float>(L.lin_acc ? L.partB_floats : 0);
  sc.max_acc = L.max_acc ? cv.take<float>(max_tree_acc_floats(a->D, a->H, L.max_parts)) : nullptr;
  sc.max_parts = L.max_acc ? L.max_parts : 0;
  sc.plan = L.plan;
  sc.sel = L.need_sel ? sel_ws : out->sel;
  sc.s_mean = L.need_sm ? sm_ws : out->s_mean;
  return sc;
}

// Parameter prep, projection + preselection, state walk and statistics of one
// E-step on stream s.  c may be NULL (no profiling).  after_B runs once B is
// complete; reserve_cu CUs are left free for work it forks.
hipError_t enqueue_estep(prosper_ctx* c, const prosper_args* a, const float* Y, const float* W,
                         const prosper_point_out* out, const prosper_acc* acc, hipStream_t s,
                         const Prepared& p, const Scratch& sc, const uint32_t* tab_act,
                         const uint32_t* tab_sgn, int64_t ns, int num_cu,
                         const StatsHook& after_B, int reserve_cu, hipStream_t a_stream) {
  const int model = a->model, prec = a->precision;
  const int64_t N = a->N;
  const int D = a->D, H = a->H, Hp = a->Hprime;
  const int Dp = padded_depth(D);
  uint8_t* flagged = out ? out->flagged : nullptr;
  float* logL = out ? out->logL : nullptr;
  uint32_t* top_mask = out ? out->top_mask : nullptr;
  float* top_q = out ? out->top_q : nullptr;
  float* Aacc = a->accumulate ? acc->A : nullptr;
  float* Bacc = a->accumulate ? acc->B : nullptr;
  double* scal = a->accumulate ? acc->scal : nullptr;
  int tree_blocks = 0;
  // PROSPER_FLAG_ZERO_ACC: the preparation kernels clear the accumulators
  const bool zero = a->accumulate && (a->flags & PROSPER_FLAG_ZERO_ACC);
  AccZero z;
  if (zero) {
    z.A = Aacc;
    z.B = Bacc;
    z.B_dh = is_max_model(model);
    z.scal = scal;
    z.vcount = model == PROSPER_DSC ? acc->vcount : nullptr;
    z.nv = model == PROSPER_DSC ? a->nvalues : 0;
  }
  hipError_t e = timed(c, "prep", s, [&] {
    hipError_t e2 = launch_theta_full(model, D, H, a->pi, a->sigma, a->theta_dev, p,
                                      sc.redo_count, s, sc.defer_count, args_beta(a),
                                      dsc_params(a), z);
    return e2 == hipSuccess ? launch_prep(model, prec, W, D, H, Dp, p, s, z) : e2;
  });
  if (e == hipSuccess)
    e = timed(c, "project_select", s, [&] {
      return launch_project_select(model, prec, Y, N, D, Dp, H, Hp, p, sc, flagged, scal, s);
    });
  if (e == hipSuccess)
    e = timed(c, is_max_model(model) ? "states_max"
                 : (model == PROSPER_DSC ? "states_dsc" : "states_lin"), s, [&] {
      if (model == PROSPER_DSC)
        return launch_states_dsc(Hp, a->gamma, N, H, ns, tab_act, tab_sgn, p, sc, logL,
                                 top_mask, top_q, a->topk, Aacc != nullptr,
                                 Aacc ? acc->vcount : nullptr, scal, s, args_beta(a), num_cu,
                                 &tree_blocks, Bacc);
      if (is_max_model(model))
        return launch_states_max(model, Hp, a->gamma, N, D, Dp, H, ns, tab_act, Y, p, sc, logL,
                                 top_mask, top_q, a->topk, Aacc, Bacc, scal, s);
      return launch_states_lin(model, Hp, a->gamma, N, H, ns, tab_act, tab_sgn, p, sc, logL,
                               top_mask, top_q, a->topk, Aacc != nullptr, Bacc, scal, num_cu,
                               &tree_blocks, s, args_beta(a), out ? out->k_mean : nullptr,
                               out ? out->res : nullptr);
    });
  if (e == hipSuccess && Aacc && !is_max_model(model)) {
    if (!after_B) {
      e = timed(c, "stats", s, [&] {
        return launch_stats(Y, N, D, H, Hp, sc, sc.plan, tree_blocks, Aacc, Bacc, s, STATS_ALL,
                            reserve_cu);
      });
    } else {
      // B first; then the hook (queues work on s that needs only B); then A,
      // on a_stream when given
      hipStream_t as = a_stream ? a_stream : s;
      e = timed(c, "stats", s, [&] {
        return launch_stats(Y, N, D, H, Hp, sc, sc.plan, tree_blocks, Aacc, Bacc, s, STATS_B,
                            reserve_cu);
      });
      if (e == hipSuccess) e = after_B(s);
      if (e == hipSuccess)
        e = timed(c, "stats_A", as, [&] {
          return launch_stats(Y, N, D, H, Hp, sc, sc.plan, tree_blocks, Aacc, Bacc, as, STATS_A,
                              reserve_cu);
        });
    }
  }
  return e;
}

}  // namespace prosper

namespace {
prosper_status mstep_entry(prosper_ctx* c, const prosper_args* a, const prosper_acc* acc,
                           const float* W_old, float* W_new, double* theta_new, void* stream,
                           const float* logL, const float* k_mean, const float* res);
}  // namespace

// ======================================================================= ABI
extern "C" {

const char* prosper_last_error(const prosper_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_tls_err.c_str();
}

prosper_status prosper_profile(prosper_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  prof_collect(c);
  c->prof_tab.clear();
  c->prof_order.clear();
  c->prof = enable != 0;
  return PROSPER_OK;
}

prosper_status prosper_profile_only(prosper_ctx* c, const char* group) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  c->prof_only = group ? group : "";
  return PROSPER_OK;
}

int32_t prosper_profile_read(prosper_ctx* c, int32_t cap, const char** names, double* total_ms,
                             int64_t* launches) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  prof_collect(c);
  int32_t i = 0;
  for (const std::string& n : c->prof_order) {
    if (i < cap) {
      // the names are string literals of this library
      static const char* known[] = {"prep",         "project_select", "states_lin",
                                    "states_max",   "states_dsc",     "stats",
                                    "stats_A",      "mstep_factor",   "mstep"};
      const char* nm = "";
      for (const char* k : known)
        if (n == k) nm = k;
      if (names) names[i] = nm;
      if (total_ms) total_ms[i] = c->prof_tab[n].ms;
      if (launches) launches[i] = c->prof_tab[n].launches;
    }
    ++i;
  }
  return i;
}

prosper_status prosper_validate_args(const prosper_args* args) {
  std::string msg;
  prosper_status st = validate(args, &msg, nullptr);
  if (st != PROSPER_OK) g_tls_err = msg;
  return st;
}

prosper_status prosper_state_count(int32_t model, int32_t Hprime, int32_t gamma, int64_t* count) {
  std::string msg;
  if (!count) return fail(nullptr, PROSPER_EINVAL, "count is NULL");
  prosper_status st = count_states(model, Hprime, gamma, count, &msg);
  if (st != PROSPER_OK) g_tls_err = msg;
  return st;
}

prosper_status prosper_state_table(int32_t model, int32_t Hprime, int32_t gamma, uint32_t* act,
                                   uint32_t* sgn, int64_t capacity) {
  int64_t n = 0;
  std::string msg;
  prosper_status st = count_states(model, Hprime, gamma, &n, &msg);
  if (st != PROSPER_OK) return fail(nullptr, st, msg);
  if (!act) return fail(nullptr, PROSPER_EINVAL, "act is NULL");
  if (capacity < n) return fail(nullptr, PROSPER_EINVAL, "capacity smaller than the state count");
  std::vector<uint32_t> a, s;
  build_table(model, Hprime, gamma, a, s);
  std::memcpy(act, a.data(), a.size() * 4);
  if (sgn) std::memcpy(sgn, s.data(), s.size() * 4);
  return PROSPER_OK;
}

prosper_status prosper_dsc_state_count(int32_t nvalues, int32_t Hprime, int32_t gamma,
                                       int64_t* count) {
  std::string msg;
  if (!count) return fail(nullptr, PROSPER_EINVAL, "count is NULL");
  prosper_status st = count_states(PROSPER_DSC, Hprime, gamma, count, &msg, nvalues);
  if (st != PROSPER_OK) g_tls_err = msg;
  return st;
}

prosper_status prosper_dsc_state_table(int32_t nvalues, int32_t Hprime, int32_t gamma,
                                       uint32_t* act, uint32_t* codes, int64_t capacity) {
  int64_t n = 0;
  std::string msg;
  prosper_status st = count_states(PROSPER_DSC, Hprime, gamma, &n, &msg, nvalues);
  if (st != PROSPER_OK) return fail(nullptr, st, msg);
  if (!act || !codes) return fail(nullptr, PROSPER_EINVAL, "act or codes is NULL");
  if (capacity < n) return fail(nullptr, PROSPER_EINVAL, "capacity smaller than the state count");
  std::vector<uint32_t> a, s;
  build_table(PROSPER_DSC, Hprime, gamma, a, s, nvalues);
  std::memcpy(act, a.data(), a.size() * 4);
  std::memcpy(codes, s.data(), s.size() * 4);
  return PROSPER_OK;
}

prosper_status prosper_ctx_create(int device, size_t workspace_bytes, prosper_ctx** out) {
  if (!out) return fail(nullptr, PROSPER_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(nullptr, PROSPER_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, PROSPER_EINVAL, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  prosper_ctx* c = new (std::nothrow) prosper_ctx();
  if (!c) return fail(nullptr, PROSPER_ENOMEM, "host allocation failed");
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  if (workspace_bytes) {
    e = ensure(c->scratch, workspace_bytes);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, PROSPER_ENOMEM, "workspace allocation failed");
    }
  }
  *out = c;
  return PROSPER_OK;
}

void prosper_ctx_destroy(prosper_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (auto& kv : c->tables) {
    hipFree(kv.second.act);
    hipFree(kv.second.sgn);
  }
  if (c->prep.p) hipFree(c->prep.p);
  if (c->scratch.p) hipFree(c->scratch.p);
  if (c->mwork.p) hipFree(c->mwork.p);
  if (c->side) hipStreamDestroy(c->side);
  if (c->ev_b) hipEventDestroy(c->ev_b);
  if (c->ev_f) hipEventDestroy(c->ev_f);
  prof_collect(c);
  for (hipEvent_t e : c->ev_free) hipEventDestroy(e);
  delete c;
}

prosper_status prosper_estep(prosper_ctx* c, const prosper_args* a, const float* Y,
                             const float* W, const prosper_point_out* out,
                             const prosper_acc* acc, void* stream) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  std::string msg;
  int64_t ns = 0;
  prosper_status st = check_estep(a, Y, W, out, acc, &msg, &ns);
  if (st != PROSPER_OK) return fail(c, st, msg);
  if (a->N == 0) return PROSPER_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");

  const int model = a->model, prec = a->precision;
  const int D = a->D, H = a->H, Hp = a->Hprime;
  const int Dp = padded_depth(D);

  Table* tab = nullptr;
  st = get_table(c, model, Hp, a->gamma, &tab, model == PROSPER_DSC ? a->nvalues : 0);
  if (st != PROSPER_OK) return st;

  e = ensure(c->prep, prep_bytes(Dp, H, prec));
  if (e != hipSuccess) return fail(c, PROSPER_ENOMEM, "workspace (parameters) allocation failed");
  Prepared p = carve_prep(c->prep.p, Dp, H, prec);

  const EstepLayout L =
      plan_estep(a, out, c->num_cu, project_defer_capacity(a->N, H, Hp, prec));
  e = ensure(c->scratch, L.bytes + 256);
  if (e != hipSuccess) return fail(c, PROSPER_ENOMEM, "workspace (per point) allocation failed");
  Scratch sc = carve_estep(c->scratch.p, L, a, out);

  if (a->accumulate) c->factor_ready = false;
  const bool factor_b = (a->flags & PROSPER_FLAG_FACTOR_B) != 0u;
  if (factor_b) {
    if (!c->side) {
      e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_f, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(c, e, "side stream for the B factor");
    }
    e = ensure(c->mwork, mstep_workspace_bytes(model, D, H));
    if (e != hipSuccess) return fail(c, PROSPER_ENOMEM, "M-step workspace allocation failed");
  }
  // after B is complete: the A statistics move to the side stream and B's
  // factorisation follows on the caller's stream (it ends after A, so the
  // join below finds A done and the M-step's solve follows the factor on the
  // same stream)
  auto after_B = [&](hipStream_t st2) -> hipError_t {
    hipError_t e2 = hipEventRecord(c->ev_b, st2);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(c->side, c->ev_b, 0);
    if (e2 == hipSuccess)
      e2 = timed(c, "mstep_factor", st2,
                 [&] { return launch_mstep_factor(model, D, H, acc->B, c->mwork.p, st2); });
    return e2;
  };
  e = enqueue_estep(c, a, Y, W, out, acc, s, p, sc, tab->act, tab->sgn, ns, c->num_cu,
                    factor_b ? StatsHook(after_B) : StatsHook(), factor_b ? 32 : 0,
                    factor_b ? c->side : nullptr);
  if (e == hipSuccess && factor_b) e = hipEventRecord(c->ev_f, c->side);
  if (e == hipSuccess && factor_b) e = hipStreamWaitEvent(s, c->ev_f, 0);
  if (e != hipSuccess) return hip_fail(c, e, "E-step launch");
  if (factor_b) {
    c->factor_ready = true;
    c->factor_B = acc->B;
    c->factor_model = model;
    c->factor_D = D;
    c->factor_H = H;
  }
  return PROSPER_OK;
}

prosper_status prosper_mstep(prosper_ctx* c, const prosper_args* a, const prosper_acc* acc,
                             const float* W_old, float* W_new, double* theta_new, void* stream) {
  return mstep_entry(c, a, acc, W_old, W_new, theta_new, stream, nullptr, nullptr, nullptr);
}

prosper_status prosper_mstep_et(prosper_ctx* c, const prosper_args* a, const prosper_acc* acc,
                                const float* logL, const float* k_mean, const float* res,
                                const float* W_old, float* W_new, double* theta_new,
                                void* stream) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  if (!a) return fail(c, PROSPER_EINVAL, "args is NULL");
  if (a->model != PROSPER_BSC && a->model != PROSPER_TSC)
    return fail(c, PROSPER_EINVAL, "the selected-points M-step is defined for BSC and TSC");
  if (a->N < 1) return fail(c, PROSPER_EINVAL, "N < 1");
  if (a->gamma < 0) return fail(c, PROSPER_EINVAL, "gamma < 0");
  if (!logL || !k_mean || !res) return fail(c, PROSPER_EINVAL, "logL, k_mean or res is NULL");
  if (!a->theta_dev && !(a->pi > 0.0 && a->pi < 1.0))
    return fail(c, PROSPER_EINVAL, "pi outside (0, 1)");
  return mstep_entry(c, a, acc, W_old, W_new, theta_new, stream, logL, k_mean, res);
}

}  // extern "C"

namespace {
// prosper_mstep, and with logL/k_mean/res the selected-points variant: its
// pi and sigma are formed before the M-step proper (which may overwrite the
// E-step's pi when theta_new aliases theta_dev) and copied in after it.
prosper_status mstep_entry(prosper_ctx* c, const prosper_args* a, const prosper_acc* acc,
                           const float* W_old, float* W_new, double* theta_new, void* stream,
                           const float* logL, const float* k_mean, const float* res) {
  if (!c) return fail(nullptr, PROSPER_EINVAL, "ctx is NULL");
  if (!a) return fail(c, PROSPER_EINVAL, "args is NULL");
  if (a->model != PROSPER_BSC && a->model != PROSPER_TSC && a->model != PROSPER_DSC &&
      !is_max_model(a->model))
    return fail(c, PROSPER_EINVAL, "unknown model");
  if (a->D < 1 || a->D > PROSPER_MAX_D || a->H < 1 || a->H > PROSPER_MAX_H)
    return fail(c, PROSPER_EINVAL, "D or H out of range");
  if (!acc || !acc->A || !acc->B || !acc->scal || !W_old || !W_new || !theta_new)
    return fail(c, PROSPER_EINVAL, "NULL pointer argument");
  const bool dsc = a->model == PROSPER_DSC;
  if (dsc && (a->nvalues < 2 || a->nvalues > PROSPER_MAX_VALUES))
    return fail(c, PROSPER_EINVAL, "DSC nvalues outside 2..8");
  if (dsc && !acc->vcount) return fail(c, PROSPER_EINVAL, "DSC M-step needs acc->vcount");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  e = ensure(c->mwork, mstep_workspace_bytes(a->model, a->D, a->H));
  if (e != hipSuccess) return fail(c, PROSPER_ENOMEM, "M-step workspace allocation failed");
  const bool reuse = c->factor_ready && c->factor_B == acc->B && c->factor_model == a->model &&
                     c->factor_D == a->D && c->factor_H == a->H;
  c->factor_ready = false;
  const bool et = logL != nullptr;
  if (et) {
    e = timed(c, "mstep", s, [&] {
      return launch_mstep_et_select(a->N, a->D, a->H, a->gamma, a->pi, a->theta_dev, logL,
                                    k_mean, res, c->mwork.p, s);
    });
    if (e != hipSuccess) return hip_fail(c, e, "M-step launch");
  }
  e = timed(c, "mstep", s, [&] {
    if (reuse)
      return launch_mstep_solve(a->model, a->D, a->H, acc->A, acc->B, acc->scal, W_old, W_new,
                                theta_new, c->mwork.p, s);
    return launch_mstep(a->model, a->D, a->H, acc->A, acc->B, acc->scal, W_old, W_new, theta_new,
                        c->mwork.p, s);
  });
  if (e == hipSuccess && dsc)
    e = launch_mstep_dsc_prior(a->H, a->nvalues, acc->scal, acc->vcount, theta_new, s);
  if (e == hipSuccess && et) e = launch_mstep_et_finish(a->D, a->H, c->mwork.p, theta_new, s);
  if (e != hipSuccess) return hip_fail(c, e, "M-step launch");
  return PROSPER_OK;
}

}  // namespace

