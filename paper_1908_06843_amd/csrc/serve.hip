// Serving runtime: E-step-only posterior inference (the API section's
// `inference`: most probable states and their posterior probabilities per
// data point) with continuous batching.
//
// One scheduler thread owns the device side.  Requests wait in a FIFO
// queue; a request is admitted as soon as (a) fewer than max_inflight
// requests are on the GPU and (b) its buffers fit in the device memory pool
// (mem_budget_bytes, first-fit).  Admitted requests are launched on the
// least-loaded of n_streams HIP streams, so requests that arrive while
// others run overlap with them on the device.  Completion is detected with
// HIP events; the scheduler copies the outputs from the pinned staging
// area into the caller's buffers, returns the memory and admits the next
// requests.  The dictionary, its derived tables (projection rows, Gram
// matrix, norms) and the state tables are built once and stay resident.
// No computation couples two requests, so a result is the same alone and
// in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "prosper_internal.hpp"

using namespace prosper;
using Clock = std::chrono::steady_clock;

namespace {

struct Pool {  // first-fit free list over [0, size)
  std::map<size_t, size_t> free_;  // offset -> length
  size_t size = 0;
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o2 = it->first + n;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  uint64_t id;
  const float* Y;
  int64_t n;
  int Hp, gamma, topk;
  prosper_point_out out;
  Clock::time_point t_submit, t_done;
  prosper_status status = PROSPER_OK;
  bool done = false;
  // device side
  size_t off = 0, bytes = 0;
  int stream = -1;
  hipEvent_t ev = nullptr;
  // layout inside the pool piece
  size_t o_Y, o_sel, o_bc, o_yy, o_sm, o_redo, o_cnt, o_logL, o_flag, o_tm, o_tq;
};

struct TableDev {
  uint32_t* act = nullptr;
  uint32_t* sgn = nullptr;
  int64_t count = 0;
};

size_t layout(Req& r, int D) {
  size_t o = 0;
  auto take = [&](size_t n) {
    o = (o + 255) & ~(size_t)255;
    size_t at = o;
    o += n;
    return at;
  };
  const size_t N = (size_t)r.n, Hp = (size_t)r.Hp, K = (size_t)r.topk;
  r.o_Y = take(N * D * 4);
  r.o_sel = take(N * Hp * 4);
  r.o_bc = take(N * Hp * 4);
  r.o_yy = take(N * 4);
  r.o_sm = take(N * Hp * 4);
  r.o_redo = take(N * 4);
  r.o_cnt = take(4);
  r.o_logL = take(N * 4);
  r.o_flag = take(N);
  r.o_tm = take(N * K * 4 * 2);
  r.o_tq = take(N * K * 4);
  return (o + 255) & ~(size_t)255;
}

}  // namespace

struct prosper_server {
  int device = 0, num_cu = 256;
  int model, D, H, Dp, prec;
  double pi, sigma;
  size_t budget;
  int max_inflight, n_streams, qcap;
  float* W = nullptr;
  void* prep_mem = nullptr;
  Prepared prep;
  int32_t* prep_redo = nullptr;
  char* dev_pool = nullptr;
  char* pin_pool = nullptr;
  Pool pool;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_load;
  std::map<std::pair<int, int>, TableDev> tables;
  std::deque<Req*> queue;
  std::vector<Req*> inflight;
  std::map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stopping = false;
  std::thread th;
  std::string err;
};

namespace {

prosper_status table_for(prosper_server* s, int Hp, int gamma, TableDev** out) {
  auto key = std::make_pair(Hp, gamma);
  auto it = s->tables.find(key);
  if (it != s->tables.end()) {
    *out = &it->second;
    return PROSPER_OK;
  }
  std::vector<uint32_t> act, sgn;
  build_table(s->model, Hp, gamma, act, sgn);
  TableDev t;
  t.count = (int64_t)act.size();
  if (hipMalloc(&t.act, act.size() * 4) != hipSuccess ||
      hipMalloc(&t.sgn, sgn.size() * 4) != hipSuccess ||
      hipMemcpy(t.act, act.data(), act.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.sgn, sgn.data(), sgn.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return PROSPER_EDEVICE;
  *out = &s->tables.emplace(key, t).first->second;
  return PROSPER_OK;
}

// Launch one admitted request (scheduler thread, lock held).
void launch(prosper_server* s, Req* r) {
  TableDev* tab = nullptr;
  prosper_status st = table_for(s, r->Hp, r->gamma, &tab);
  if (st != PROSPER_OK) {
    r->status = st;
    return;
  }
  int best = 0;
  for (int i = 1; i < s->n_streams; ++i)
    if (s->stream_load[i] < s->stream_load[best]) best = i;
  r->stream = best;
  s->stream_load[best]++;
  hipStream_t stm = s->streams[best];
  char* dev = s->dev_pool + r->off;
  char* pin = s->pin_pool + r->off;
  std::memcpy(pin + r->o_Y, r->Y, (size_t)r->n * s->D * 4);
  hipError_t e = hipMemcpyAsync(dev + r->o_Y, pin + r->o_Y, (size_t)r->n * s->D * 4,
                                hipMemcpyHostToDevice, stm);
  Scratch sc;
  sc.sel = reinterpret_cast<int32_t*>(dev + r->o_sel);
  sc.bc = reinterpret_cast<float*>(dev + r->o_bc);
  sc.yy = reinterpret_cast<float*>(dev + r->o_yy);
  sc.s_mean = reinterpret_cast<float*>(dev + r->o_sm);
  sc.redo_list = reinterpret_cast<int32_t*>(dev + r->o_redo);
  sc.redo_count = reinterpret_cast<int32_t*>(dev + r->o_cnt);
  sc.ss = nullptr;
  sc.partA = sc.partB = nullptr;
  float* logL = reinterpret_cast<float*>(dev + r->o_logL);
  uint8_t* flag = reinterpret_cast<uint8_t*>(dev + r->o_flag);
  uint32_t* tm = r->topk ? reinterpret_cast<uint32_t*>(dev + r->o_tm) : nullptr;
  float* tq = r->topk ? reinterpret_cast<float*>(dev + r->o_tq) : nullptr;
  if (e == hipSuccess) e = hipMemsetAsync(sc.redo_count, 0, 4, stm);
  if (e == hipSuccess)
    e = launch_estep_core(s->model, s->prec, reinterpret_cast<const float*>(dev + r->o_Y), r->n,
                          s->D, s->H, r->Hp, r->gamma, tab->count, tab->act, tab->sgn, s->prep,
                          sc, flag, logL, tm, tq, r->topk, nullptr, nullptr, nullptr, s->num_cu,
                          stm);
  // outputs back to the pinned area
  auto d2h = [&](size_t o, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(pin + o, dev + o, n, hipMemcpyDeviceToHost, stm);
  };
  const size_t N = (size_t)r->n, Hp = (size_t)r->Hp, K = (size_t)r->topk;
  const size_t tmw = (s->model == PROSPER_TSC) ? 2 : 1;
  if (r->out.sel) d2h(r->o_sel, N * Hp * 4);
  if (r->out.s_mean) d2h(r->o_sm, N * Hp * 4);
  if (r->out.logL) d2h(r->o_logL, N * 4);
  if (r->out.flagged) d2h(r->o_flag, N);
  if (r->out.top_mask && K) d2h(r->o_tm, N * K * 4 * tmw);
  if (r->out.top_q && K) d2h(r->o_tq, N * K * 4);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r->ev, stm);
  if (e != hipSuccess) {
    s->err = std::string("serve launch: ") + hipGetErrorString(e);
    r->status = PROSPER_EDEVICE;
  }
}

void finish(prosper_server* s, Req* r) {
  const char* pin = s->pin_pool + r->off;
  const size_t N = (size_t)r->n, Hp = (size_t)r->Hp, K = (size_t)r->topk;
  const size_t tmw = (s->model == PROSPER_TSC) ? 2 : 1;
  if (r->status == PROSPER_OK) {
    if (r->out.sel) std::memcpy(r->out.sel, pin + r->o_sel, N * Hp * 4);
    if (r->out.s_mean) std::memcpy(r->out.s_mean, pin + r->o_sm, N * Hp * 4);
    if (r->out.logL) std::memcpy(r->out.logL, pin + r->o_logL, N * 4);
    if (r->out.flagged) std::memcpy(r->out.flagged, pin + r->o_flag, N);
    if (r->out.top_mask && K) std::memcpy(r->out.top_mask, pin + r->o_tm, N * K * 4 * tmw);
    if (r->out.top_q && K) std::memcpy(r->out.top_q, pin + r->o_tq, N * K * 4);
  }
  if (r->ev) hipEventDestroy(r->ev);
  r->ev = nullptr;
  if (r->stream >= 0) s->stream_load[r->stream]--;
  s->pool.release(r->off, r->bytes);
  r->t_done = Clock::now();
  r->done = true;
}

void scheduler(prosper_server* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // admit in arrival order while slots and memory allow
    while (!s->queue.empty() && (int)s->inflight.size() < s->max_inflight) {
      Req* r = s->queue.front();
      size_t off = 0;
      if (!s->pool.alloc(r->bytes, &off)) break;
      s->queue.pop_front();
      r->off = off;
      launch(s, r);
      if (r->status != PROSPER_OK) {
        finish(s, r);
        s->cv_done.notify_all();
        continue;
      }
      s->inflight.push_back(r);
    }
    // retire completed requests
    bool any = false;
    for (size_t i = 0; i < s->inflight.size();) {
      Req* r = s->inflight[i];
      hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) r->status = PROSPER_EDEVICE;
      finish(s, r);
      s->inflight.erase(s->inflight.begin() + i);
      any = true;
    }
    if (any) s->cv_done.notify_all();
    if (s->stopping && s->queue.empty() && s->inflight.empty()) break;
    if (s->inflight.empty() && s->queue.empty()) {
      s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
    } else if (!any) {
      // requests on the GPU: poll their events again shortly
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

prosper_status prosper_serve(prosper_ctx* ctx, const float* W, int32_t W_on_device,
                             int32_t model, int32_t D, int32_t H, double pi, double sigma,
                             int32_t precision, size_t mem_budget_bytes, int32_t max_inflight,
                             int32_t n_streams, int32_t queue_capacity, prosper_server** out) {
  if (!ctx || !W || !out) return PROSPER_EINVAL;
  *out = nullptr;
  if (model != PROSPER_BSC && model != PROSPER_TSC && model != PROSPER_MCA) return PROSPER_EINVAL;
  if (precision != PROSPER_FP32 && precision != PROSPER_BF16) return PROSPER_EINVAL;
  if (D < 1 || D > PROSPER_MAX_D || H < 1 || H > PROSPER_MAX_H) return PROSPER_EINVAL;
  if (!(pi > 0.0 && pi < 1.0) || !(sigma > 0.0)) return PROSPER_EINVAL;
  if (max_inflight < 1 || n_streams < 1 || n_streams > 8 || queue_capacity < 1 ||
      mem_budget_bytes < 4096)
    return PROSPER_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PROSPER_EDEVICE;
  prosper_server* s = new (std::nothrow) prosper_server();
  if (!s) return PROSPER_ENOMEM;
  s->device = dev;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    s->num_cu = prop.multiProcessorCount;
  s->model = model;
  s->D = D;
  s->H = H;
  s->Dp = padded_depth(D);
  s->prec = precision;
  s->pi = pi;
  s->sigma = sigma;
  s->budget = mem_budget_bytes;
  s->max_inflight = max_inflight;
  s->n_streams = n_streams;
  s->qcap = queue_capacity;
  hipError_t e = hipMalloc(&s->W, (size_t)D * H * 4);
  if (e == hipSuccess)
    e = hipMemcpy(s->W, W, (size_t)D * H * 4,
                  W_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&s->prep_mem, prep_bytes(s->Dp, H, precision));
  if (e == hipSuccess) e = hipMalloc(&s->prep_redo, 4);
  if (e == hipSuccess) e = hipMalloc(&s->dev_pool, mem_budget_bytes);
  if (e == hipSuccess) e = hipHostMalloc(&s->pin_pool, mem_budget_bytes, hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < n_streams; ++i) {
    hipStream_t st;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(st);
  }
  if (e == hipSuccess) {
    s->prep = carve_prep(s->prep_mem, s->Dp, H, precision);
    e = launch_theta_full(model, D, H, pi, sigma, nullptr, s->prep, s->prep_redo, s->streams[0]);
    if (e == hipSuccess) e = launch_prep(model, precision, s->W, D, H, s->Dp, s->prep, s->streams[0]);
    if (e == hipSuccess) e = hipStreamSynchronize(s->streams[0]);
  }
  if (e != hipSuccess) {
    prosper_serve_stop(s);
    return PROSPER_EDEVICE;
  }
  s->pool.init(mem_budget_bytes);
  s->stream_load.assign(n_streams, 0);
  s->th = std::thread(scheduler, s);
  *out = s;
  return PROSPER_OK;
}

prosper_status prosper_serve_submit(prosper_server* s, const float* Y_host, int64_t npatches,
                                    int32_t Hprime, int32_t gamma, int32_t topk,
                                    const prosper_point_out* out_host, uint64_t* req_id) {
  if (!s || !req_id || npatches < 1 || !Y_host) return PROSPER_EINVAL;
  prosper_args a{};
  a.model = s->model;
  a.precision = s->prec;
  a.N = npatches;
  a.D = s->D;
  a.H = s->H;
  a.Hprime = Hprime;
  a.gamma = gamma;
  a.pi = s->pi;
  a.sigma = s->sigma;
  a.topk = topk;
  if (prosper_validate_args(&a) != PROSPER_OK) return PROSPER_EINVAL;
  Req* r = new (std::nothrow) Req();
  if (!r) return PROSPER_ENOMEM;
  r->Y = Y_host;
  r->n = npatches;
  r->Hp = Hprime;
  r->gamma = gamma;
  r->topk = topk;
  if (out_host) r->out = *out_host;
  r->bytes = layout(*r, s->D);
  if (r->bytes > s->budget) {
    delete r;
    return PROSPER_EINVAL;
  }
  std::lock_guard<std::mutex> g(s->mu);
  if ((int)s->queue.size() >= s->qcap || s->stopping) {
    delete r;
    return PROSPER_EBUSY;
  }
  r->id = s->next_id++;
  r->t_submit = Clock::now();
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  *req_id = r->id;
  s->cv_work.notify_one();
  return PROSPER_OK;
}

prosper_status prosper_serve_wait(prosper_server* s, uint64_t id, int64_t timeout_us,
                                  double* latency_ms) {
  if (!s) return PROSPER_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return PROSPER_ENOTFOUND;
  Req* r = it->second;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                  [&] { return r->done; })) {
    return PROSPER_ETIMEDOUT;
  }
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  prosper_status st = r->status;
  s->reqs.erase(it);
  delete r;
  return st;
}

prosper_status prosper_serve_stop(prosper_server* s) {
  if (!s) return PROSPER_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->reqs) delete kv.second;
  for (auto& kv : s->tables) {
    hipFree(kv.second.act);
    hipFree(kv.second.sgn);
  }
  for (hipStream_t st : s->streams) hipStreamDestroy(st);
  if (s->W) hipFree(s->W);
  if (s->prep_mem) hipFree(s->prep_mem);
  if (s->prep_redo) hipFree(s->prep_redo);
  if (s->dev_pool) hipFree(s->dev_pool);
  if (s->pin_pool) hipHostFree(s->pin_pool);
  delete s;
  return PROSPER_OK;
}

}  // extern "C"
