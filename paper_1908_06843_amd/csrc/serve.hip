// Serving runtime: E-step-only posterior inference (the API section's
// `inference`: most probable states and their posterior probabilities per
// data point) with continuous batching.
//
// One scheduler thread owns the device side.  Requests wait in a FIFO
// queue.  Whenever fewer than max_inflight batches are on the GPU, the
// scheduler forms a batch from the head of the queue: the head request plus
// the queued requests with the same (H', gamma, topk), up to a row limit,
// whose combined buffers fit in the device memory pool (mem_budget_bytes,
// first-fit); a request that does not fit waits for memory to be returned.
// A batch costs one staging copy, one set of kernel launches and one copy
// back per output, and runs on the least-loaded of n_streams HIP streams,
// so batches formed while others run overlap with them on the device.
// Completion is detected with HIP events; the scheduler then copies each
// member's rows from the pinned staging area into its caller's buffers,
// returns the memory and forms the next batches.  The dictionary, its
// derived tables (projection rows, Gram matrix, norms) and the state tables
// are built once and stay resident.  Every output of a point depends only on
// that point and the dictionary, so a result is the same alone and in any
// batch or mix.
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
  // stage times: submit, batch launch begins / returns, completion seen by
  // the scheduler, outputs delivered; GPU time of its batch (events)
  Clock::time_point t_submit, t_launch, t_launched, t_seen, t_done;
  float gpu_ms = 0.0f;
  prosper_status status = PROSPER_OK;
  bool done = false;
  int64_t row0 = 0;  // first row inside its batch
  // pinned copy of Y made by the submitting thread (ingress pool), if any
  size_t in_off = 0, in_bytes = 0;
  bool staged = false;
};

struct Batch {
  std::vector<Req*> reqs;
  int Hp = 0, gamma = 0, topk = 0;
  int64_t n = 0;
  size_t off = 0, bytes = 0;
  int stream = -1;
  hipEvent_t ev = nullptr;        // end of the batch's work on its stream
  hipEvent_t ev_start = nullptr;  // start of it
  prosper_status status = PROSPER_OK;
  bool w_sel = false, w_sm = false, w_logL = false, w_flag = false, w_tm = false, w_tq = false;
  // layout inside the pool piece
  size_t o_Y, o_sel, o_bc, o_yy, o_sm, o_redo, o_cnt, o_logL, o_flag, o_tm, o_tq;
  size_t o_end;  // end of the outputs (o_sel .. o_end holds all of them)
};

struct TableDev {
  uint32_t* act = nullptr;
  uint32_t* sgn = nullptr;
  int64_t count = 0;
};

// Device bytes of n rows with H' candidates and topk states (one piece).
size_t layout_bytes(int64_t n, int Hp, int topk, int D, Batch* b) {
  size_t o = 0;
  auto take = [&](size_t m) {
    o = (o + 255) & ~(size_t)255;
    size_t at = o;
    o += m;
    return at;
  };
  const size_t N = (size_t)n, H1 = (size_t)Hp, K = (size_t)topk;
  // inputs and scratch first, then the outputs back to back, so that one
  // copy returns all of them
  const size_t oY = take(N * D * 4), obc = take(N * H1 * 4), oyy = take(N * 4),
               oredo = take(N * 4), ocnt = take(4), osel = take(N * H1 * 4),
               osm = take(N * H1 * 4), ologL = take(N * 4), oflag = take(N),
               otm = take(N * K * 4 * 2), otq = take(N * K * 4);
  if (b) b->o_end = otq + N * K * 4;
  if (b) {
    b->o_Y = oY;
    b->o_sel = osel;
    b->o_bc = obc;
    b->o_yy = oyy;
    b->o_sm = osm;
    b->o_redo = oredo;
    b->o_cnt = ocnt;
    b->o_logL = ologL;
    b->o_flag = oflag;
    b->o_tm = otm;
    b->o_tq = otq;
  }
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
  char* in_pool = nullptr;  // pinned ingress area for request inputs
  Pool pool;
  Pool in_free;             // shared with submit: lock held
  std::vector<hipStream_t> streams;
  std::vector<int> stream_load;
  std::map<std::pair<int, int>, TableDev> tables;
  std::deque<Req*> queue;
  std::vector<Batch*> inflight;     // scheduler thread only
  std::vector<hipEvent_t> ev_pool;  // scheduler thread only
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

// Rows of one batch at most (unless its head request alone is larger): keeps
// the wait of a small request behind the big ones it is batched with short.
static constexpr int64_t BATCH_ROWS = 2048;

// Form the next batch from the queue (lock held).  Returns nullptr when the
// queue is empty or the head request does not fit in the free memory.
Batch* form_batch(prosper_server* s) {
  if (s->queue.empty()) return nullptr;
  Req* head = s->queue.front();
  Batch* b = new (std::nothrow) Batch();
  if (!b) return nullptr;
  b->Hp = head->Hp;
  b->gamma = head->gamma;
  b->topk = head->topk;
  std::vector<size_t> pick;  // queue positions, in order
  int64_t rows = 0;
  const int64_t limit = std::max<int64_t>(head->n, BATCH_ROWS);
  for (size_t i = 0; i < s->queue.size() && i < 64; ++i) {
    Req* r = s->queue[i];
    if (r->Hp != b->Hp || r->gamma != b->gamma || r->topk != b->topk) continue;
    if (rows + r->n > limit) break;
    pick.push_back(i);
    rows += r->n;
  }
  // largest prefix of the picks that fits in the pool
  size_t off = 0;
  while (!pick.empty()) {
    int64_t n = 0;
    for (size_t i : pick) n += s->queue[i]->n;
    const size_t bytes = layout_bytes(n, b->Hp, b->topk, s->D, b);
    if (s->pool.alloc(bytes, &off)) {
      b->n = n;
      b->bytes = bytes;
      b->off = off;
      break;
    }
    pick.pop_back();
  }
  if (pick.empty()) {
    delete b;
    return nullptr;
  }
  int64_t row = 0;
  for (size_t i : pick) {
    Req* r = s->queue[i];
    r->row0 = row;
    row += r->n;
    b->reqs.push_back(r);
    b->w_sel |= r->out.sel != nullptr;
    b->w_sm |= r->out.s_mean != nullptr;
    b->w_logL |= r->out.logL != nullptr;
    b->w_flag |= r->out.flagged != nullptr;
    b->w_tm |= r->out.top_mask != nullptr && r->topk > 0;
    b->w_tq |= r->out.top_q != nullptr && r->topk > 0;
  }
  for (size_t k = pick.size(); k-- > 0;) s->queue.erase(s->queue.begin() + pick[k]);
  return b;
}

// Launch one batch (scheduler thread; the batch's pool piece is its own, so
// no lock is needed).
void launch(prosper_server* s, Batch* b) {
  TableDev* tab = nullptr;
  prosper_status st = table_for(s, b->Hp, b->gamma, &tab);
  if (st != PROSPER_OK) {
    b->status = st;
    return;
  }
  int best = 0;
  for (int i = 1; i < s->n_streams; ++i)
    if (s->stream_load[i] < s->stream_load[best]) best = i;
  b->stream = best;
  s->stream_load[best]++;
  hipStream_t stm = s->streams[best];
  // timing events of the batch (a pool of them is kept; default flags, so
  // that the batch's GPU time can be read)
  hipError_t e = hipSuccess;
  for (hipEvent_t* evp : {&b->ev_start, &b->ev}) {
    if (e != hipSuccess) break;
    if (!s->ev_pool.empty()) {
      *evp = s->ev_pool.back();
      s->ev_pool.pop_back();
    } else {
      e = hipEventCreate(evp);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(b->ev_start, stm);
  char* dev = s->dev_pool + b->off;
  char* pin = s->pin_pool + b->off;
  const size_t row_bytes = (size_t)s->D * 4;
  bool all_staged = true;
  for (Req* r : b->reqs) all_staged &= r->staged;
  if (e != hipSuccess) {
  } else if (all_staged) {
    // inputs were copied to pinned memory by the submitting threads
    for (Req* r : b->reqs)
      if (e == hipSuccess)
        e = hipMemcpyAsync(dev + b->o_Y + (size_t)r->row0 * row_bytes, s->in_pool + r->in_off,
                           (size_t)r->n * row_bytes, hipMemcpyHostToDevice, stm);
  } else {
    for (Req* r : b->reqs) {
      const char* src = r->staged ? s->in_pool + r->in_off : reinterpret_cast<const char*>(r->Y);
      std::memcpy(pin + b->o_Y + (size_t)r->row0 * row_bytes, src, (size_t)r->n * row_bytes);
    }
    e = hipMemcpyAsync(dev + b->o_Y, pin + b->o_Y, (size_t)b->n * row_bytes,
                       hipMemcpyHostToDevice, stm);
  }
  Scratch sc;
  sc.sel = reinterpret_cast<int32_t*>(dev + b->o_sel);
  sc.bc = reinterpret_cast<float*>(dev + b->o_bc);
  sc.yy = reinterpret_cast<float*>(dev + b->o_yy);
  sc.s_mean = reinterpret_cast<float*>(dev + b->o_sm);
  sc.redo_list = reinterpret_cast<int32_t*>(dev + b->o_redo);
  sc.redo_count = reinterpret_cast<int32_t*>(dev + b->o_cnt);
  sc.ss = nullptr;
  sc.partA = sc.partB = nullptr;
  float* logL = reinterpret_cast<float*>(dev + b->o_logL);
  uint8_t* flag = reinterpret_cast<uint8_t*>(dev + b->o_flag);
  uint32_t* tm = b->topk ? reinterpret_cast<uint32_t*>(dev + b->o_tm) : nullptr;
  float* tq = b->topk ? reinterpret_cast<float*>(dev + b->o_tq) : nullptr;
  if (e == hipSuccess) e = hipMemsetAsync(sc.redo_count, 0, 4, stm);
  if (e == hipSuccess)
    e = launch_estep_core(s->model, s->prec, reinterpret_cast<const float*>(dev + b->o_Y), b->n,
                          s->D, s->H, b->Hp, b->gamma, tab->count, tab->act, tab->sgn, s->prep,
                          sc, flag, logL, tm, tq, b->topk, nullptr, nullptr, nullptr, s->num_cu,
                          stm);
  // outputs back to the pinned area: one copy over the contiguous output
  // span (a few tens of bytes per row; fewer API calls on the scheduler
  // thread matter more than the unwanted bytes)
  if (e == hipSuccess && (b->w_sel || b->w_sm || b->w_logL || b->w_flag || b->w_tm || b->w_tq))
    e = hipMemcpyAsync(pin + b->o_sel, dev + b->o_sel, b->o_end - b->o_sel,
                       hipMemcpyDeviceToHost, stm);
  if (e == hipSuccess) e = hipEventRecord(b->ev, stm);
  if (e != hipSuccess) {
    s->err = std::string("serve launch: ") + hipGetErrorString(e);
    b->status = PROSPER_EDEVICE;
  }
}

// Copy each member's rows of a completed batch to its caller's buffers and
// return the batch's stream slot, event and memory (scheduler thread, no lock).
void deliver(prosper_server* s, Batch* b) {
  const char* pin = s->pin_pool + b->off;
  const size_t Hp = (size_t)b->Hp, K = (size_t)b->topk;
  const size_t tmw = (s->model == PROSPER_TSC) ? 2 : 1;
  for (Req* r : b->reqs) {
    r->status = b->status;
    if (b->status != PROSPER_OK) continue;
    const size_t n = (size_t)r->n, r0 = (size_t)r->row0;
    if (r->out.sel) std::memcpy(r->out.sel, pin + b->o_sel + r0 * Hp * 4, n * Hp * 4);
    if (r->out.s_mean) std::memcpy(r->out.s_mean, pin + b->o_sm + r0 * Hp * 4, n * Hp * 4);
    if (r->out.logL) std::memcpy(r->out.logL, pin + b->o_logL + r0 * 4, n * 4);
    if (r->out.flagged) std::memcpy(r->out.flagged, pin + b->o_flag + r0, n);
    if (r->out.top_mask && K)
      std::memcpy(r->out.top_mask, pin + b->o_tm + r0 * K * 4 * tmw, n * K * 4 * tmw);
    if (r->out.top_q && K) std::memcpy(r->out.top_q, pin + b->o_tq + r0 * K * 4, n * K * 4);
  }
  if (b->ev) s->ev_pool.push_back(b->ev);
  if (b->ev_start) s->ev_pool.push_back(b->ev_start);
  b->ev = b->ev_start = nullptr;
  if (b->stream >= 0) s->stream_load[b->stream]--;
  s->pool.release(b->off, b->bytes);
}

// The scheduler.  Only the queue, the request table and the done flags are
// shared with submit/wait and need the lock (forming a batch takes its memory
// under the lock too); staging copies, launches, completion queries and
// output copies run without it, so callers are never blocked behind them.
// While batches are on the GPU it polls their events without sleeping (a
// sleep would add the timer slack to every latency).
void scheduler(prosper_server* s) {
  hipSetDevice(s->device);
  std::vector<Batch*> admit, done;
  while (true) {
    admit.clear();
    done.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->inflight.empty() && s->queue.empty()) {
        if (s->stopping) break;
        s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
        if (s->stopping && s->queue.empty()) break;
      }
      while ((int)(s->inflight.size() + admit.size()) < s->max_inflight) {
        Batch* b = form_batch(s);
        if (!b) break;
        admit.push_back(b);
      }
    }
    for (Batch* b : admit) {
      const Clock::time_point t0 = Clock::now();
      for (Req* r : b->reqs) r->t_launch = t0;
      launch(s, b);
      const Clock::time_point t1 = Clock::now();
      for (Req* r : b->reqs) r->t_launched = t1;
      if (b->status != PROSPER_OK) done.push_back(b);
      else s->inflight.push_back(b);
    }
    for (size_t i = 0; i < s->inflight.size();) {
      Batch* b = s->inflight[i];
      const hipError_t q = hipEventQuery(b->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) b->status = PROSPER_EDEVICE;
      const Clock::time_point t_seen = Clock::now();
      float gpu_ms = 0.0f;
      if (q == hipSuccess && hipEventElapsedTime(&gpu_ms, b->ev_start, b->ev) != hipSuccess)
        gpu_ms = 0.0f;
      for (Req* r : b->reqs) {
        r->t_seen = t_seen;
        r->gpu_ms = gpu_ms;
      }
      done.push_back(b);
      s->inflight.erase(s->inflight.begin() + i);
    }
    for (Batch* b : done) deliver(s, b);
    if (!done.empty()) {
      const Clock::time_point now = Clock::now();
      {
        std::lock_guard<std::mutex> g(s->mu);
        for (Batch* b : done)
          for (Req* r : b->reqs) {
            if (r->staged) s->in_free.release(r->in_off, r->in_bytes);
            r->staged = false;
            r->t_done = now;
            r->done = true;
          }
      }
      s->cv_done.notify_all();
      for (Batch* b : done) delete b;
    } else if (admit.empty()) {
      std::this_thread::yield();
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
  if (model != PROSPER_BSC && model != PROSPER_TSC && !is_max_model(model)) return PROSPER_EINVAL;
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
  if (e == hipSuccess) e = hipHostMalloc(&s->in_pool, mem_budget_bytes, hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < n_streams; ++i) {
    hipStream_t st;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(st);
  }
  // the batches' start and end events, made here rather than on the
  // scheduler thread (creating one there delays every request behind it)
  for (int i = 0; e == hipSuccess && i < 2 * max_inflight + 2; ++i) {
    hipEvent_t ev;
    e = hipEventCreate(&ev);
    if (e == hipSuccess) s->ev_pool.push_back(ev);
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
  s->in_free.init(mem_budget_bytes);
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
  if (layout_bytes(npatches, Hprime, topk, s->D, nullptr) > s->budget) {
    delete r;
    return PROSPER_EINVAL;
  }
  const Clock::time_point t_submit = Clock::now();
  // copy the input to the pinned ingress area on this thread when it has
  // room (otherwise the scheduler stages it when the request is launched)
  const size_t in_bytes = (size_t)npatches * s->D * 4;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if ((int)s->queue.size() >= s->qcap || s->stopping) {
      delete r;
      return PROSPER_EBUSY;
    }
    r->staged = s->in_free.alloc(in_bytes, &r->in_off);
    if (r->staged) r->in_bytes = in_bytes;
  }
  if (r->staged) std::memcpy(s->in_pool + r->in_off, Y_host, in_bytes);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stopping) {
    if (r->staged) s->in_free.release(r->in_off, r->in_bytes);
    delete r;
    return PROSPER_EBUSY;
  }
  r->id = s->next_id++;
  r->t_submit = t_submit;
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  *req_id = r->id;
  s->cv_work.notify_one();
  return PROSPER_OK;
}

static prosper_status serve_wait(prosper_server* s, uint64_t id, int64_t timeout_us,
                                 double* latency_ms, double* stages_ms) {
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
  auto ms = [](Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  if (latency_ms) *latency_ms = ms(r->t_submit, r->t_done);
  if (stages_ms) {
    const bool ran = r->t_launch.time_since_epoch().count() != 0;
    stages_ms[0] = ran ? ms(r->t_submit, r->t_launch) : 0.0;
    stages_ms[1] = ran ? ms(r->t_launch, r->t_launched) : 0.0;
    stages_ms[2] = ran ? ms(r->t_launched, r->t_seen) : 0.0;
    stages_ms[3] = r->gpu_ms;
    stages_ms[4] = ran ? ms(r->t_seen, r->t_done) : 0.0;
    stages_ms[5] = ms(r->t_submit, r->t_done);
  }
  prosper_status st = r->status;
  s->reqs.erase(it);
  delete r;
  return st;
}

prosper_status prosper_serve_wait(prosper_server* s, uint64_t id, int64_t timeout_us,
                                  double* latency_ms) {
  return serve_wait(s, id, timeout_us, latency_ms, nullptr);
}

prosper_status prosper_serve_wait_stages(prosper_server* s, uint64_t id, int64_t timeout_us,
                                         double* stages_ms) {
  return serve_wait(s, id, timeout_us, nullptr, stages_ms);
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
  for (hipEvent_t ev : s->ev_pool) hipEventDestroy(ev);
  if (s->W) hipFree(s->W);
  if (s->prep_mem) hipFree(s->prep_mem);
  if (s->prep_redo) hipFree(s->prep_redo);
  if (s->dev_pool) hipFree(s->dev_pool);
  if (s->pin_pool) hipHostFree(s->pin_pool);
  if (s->in_pool) hipHostFree(s->in_pool);
  delete s;
  return PROSPER_OK;
}

}  // extern "C"
