// The E-step entry point that allocates nothing (prosper_estep_static): one
// file-scope device array per GPU holds every intermediate of the call, its
// device address is looked up once per device, and a kernel writes the
// canonical state table into it (so the call needs no host-to-device copy
// either).  The launch sequence is prosper_estep's.
#include <mutex>
#include <string>

#include "dev_common.hpp"
#include "prosper_internal.hpp"

namespace prosper {

static constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static constexpr int STATIC_MAX_DEVICES = 64;

// Only its device address (from hipGetSymbolAddress) is ever used by host code.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

static size_t static_scratch_bytes() { return STATIC_SCRATCH_BYTES; }

static void* static_scratch(int device, hipError_t* err) {
  static std::mutex mu;
  static void* ptr[STATIC_MAX_DEVICES] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= STATIC_MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!ptr[device]) {
    void* p = nullptr;
    // the caller has made `device` current
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    ptr[device] = p;
  }
  *err = hipSuccess;
  return ptr[device];
}

__device__ __forceinline__ uint64_t binom_dev(int n, int k) {
  if (k < 0 || k > n) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

// State t of the canonical order: number of actives k ascending, then the
// lexicographic rank of the slot tuple among the k-subsets of the H' slots,
// then the value code of the support counting up in base `radix` (1: BSC,
// MCA, MMCA; 2: TSC; V-1: DSC): TSC bit i of the code is the sign of the
// i-th active slot (set = -1, stored as a mask); DSC digit i plus one is the
// value code of the i-th active slot (stored in bits 3i .. 3i+2).
__global__ __launch_bounds__(256) void k_build_table(int radix, int dsc, int Hp, int gamma,
                                                     int64_t ns, uint32_t* __restrict__ act,
                                                     uint32_t* __restrict__ sgn) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ns) return;
  int64_t r = t;
  int k = 0;
  int64_t pw = 1;  // radix^k
  for (; k <= gamma; ++k) {
    const int64_t cnt = (int64_t)binom_dev(Hp, k) * pw;
    if (r < cnt) break;
    r -= cnt;
    pw *= radix;
  }
  const uint64_t code = (uint64_t)(r % pw);
  uint64_t comb = (uint64_t)(r / pw);
  uint64_t digits = code;
  uint32_t a = 0u, s = 0u;
  int x = 0;
  for (int i = 0; i < k; ++i) {
    while (true) {
      const uint64_t c = binom_dev(Hp - x - 1, k - i - 1);  // tuples whose i-th slot is x
      if (comb < c) break;
      comb -= c;
      ++x;
    }
    a |= 1u << x;
    const uint32_t dg = (uint32_t)(digits % (uint64_t)radix);
    digits /= (uint64_t)radix;
    if (dsc) s |= (1u + dg) << (3 * i);
    else if (dg) s |= 1u << x;
    ++x;
  }
  act[t] = a;
  sgn[t] = s;
}

static hipError_t launch_build_table(int model, int nv, int Hp, int gamma, int64_t ns,
                                     uint32_t* act, uint32_t* sgn, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  const int radix = model == PROSPER_TSC ? 2 : (model == PROSPER_DSC ? nv - 1 : 1);
  hipLaunchKernelGGL(k_build_table, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, radix,
                     model == PROSPER_DSC ? 1 : 0, Hp, gamma, ns, act, sgn);
  return hipGetLastError();
}

static prosper_status hip_error(hipError_t e, const char* where) {
  return set_error(PROSPER_EDEVICE, std::string(where) + ": " + hipGetErrorName(e) + " (" +
                                        hipGetErrorString(e) + ")");
}

}  // namespace prosper

using namespace prosper;

extern "C" {

prosper_status prosper_estep_static(const prosper_args* a, const float* Y, const float* W,
                                    const prosper_point_out* out, const prosper_acc* acc,
                                    void* stream) {
  std::string msg;
  int64_t ns = 0;
  prosper_status st = check_estep(a, Y, W, out, acc, &msg, &ns);
  if (st != PROSPER_OK) return set_error(st, msg);
  if (a->flags & PROSPER_FLAG_FACTOR_B)
    return set_error(PROSPER_EINVAL, "PROSPER_FLAG_FACTOR_B needs a context (prosper_estep)");
  if (a->N == 0) return PROSPER_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || ncu <= 0) return hip_error(e, "device attributes");
  char* base = reinterpret_cast<char*>(static_scratch(dev, &e));
  if (!base) return hip_error(e, "static scratch address");
  const size_t cap = static_scratch_bytes();
  // statistics partials for at most 32 workgroups keep the layout small
  const int ncu_s = ncu < 32 ? ncu : 32;
  const int H = a->H, Hp = a->Hprime, Dp = padded_depth(a->D);
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t tab_b = up((size_t)ns * 4);
  const size_t fixed = 2 * tab_b + up(prep_bytes(Dp, H, a->precision));
  EstepLayout L = plan_estep(a, out, ncu_s, 0);
  if (fixed + L.bytes + 256 > cap)
    return set_error(PROSPER_EINVAL,
                     "input needs " + std::to_string(fixed + L.bytes + 256) +
                         " bytes of scratch; prosper_estep_static holds " + std::to_string(cap));
  // the projection's deferral list takes what is left (a shorter list only
  // keeps more exact selections inside the projection workgroups)
  const size_t per_entry = (size_t)(L.Hpad + 8) * 4;
  const int64_t room =
      ((int64_t)cap - (int64_t)fixed - (int64_t)L.bytes - 512) / (int64_t)per_entry;
  int64_t dcap = project_defer_capacity(a->N, H, Hp, a->precision);
  if (dcap > room) dcap = room > 0 ? room : 0;
  L = plan_estep(a, out, ncu_s, (int)dcap);
  if (fixed + L.bytes + 256 > cap) L = plan_estep(a, out, ncu_s, 0);
  uint32_t* act = reinterpret_cast<uint32_t*>(base);
  uint32_t* sgn = reinterpret_cast<uint32_t*>(base + tab_b);
  Prepared p = carve_prep(base + 2 * tab_b, Dp, H, a->precision);
  Scratch sc = carve_estep(base + fixed, L, a, out);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  e = launch_build_table(is_max_model(a->model) ? PROSPER_BSC : a->model, a->nvalues, Hp,
                         a->gamma, ns, act, sgn, s);
  if (e == hipSuccess)
    e = enqueue_estep(nullptr, a, Y, W, out, acc, s, p, sc, act, sgn, ns, ncu_s, StatsHook(), 0);
  if (e != hipSuccess) return hip_error(e, "E-step launch");
  return PROSPER_OK;
}

}  // extern "C"
