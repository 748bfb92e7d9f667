// Host runtime of libdf3c: argument validation, class binning, planning and
// launches behind the C ABI of include/df3c.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/df3c.h"
#include "registry.hpp"

namespace df3c {
namespace {

constexpr int NCLS = NLP * NLA * NLA;  // class id = (LP * 5 + la) * 5 + lb
constexpr int MAX_DEV = 64;

constexpr int NBRANCH = 4;  // concurrent branches of the batched persistent schedule
struct DevState {
  bool ready = false;
  const double *boys = nullptr;  // the code object's Boys table on this device
  char *scratch = nullptr;       // this device's copy of the no-allocation workspace
  int ncu = 0;
  // side streams and fork/join events of the batched schedule's branches
  // (created on first use, default priority)
  bool branches = false;
  hipStream_t side[NBRANCH - 1] = {};
  hipEvent_t fork = nullptr, join[NBRANCH - 1] = {};
};
DevState g_dev[MAX_DEV];
std::mutex g_mu;
ClassInfo g_cls[NLP][NLA][NLA];
GradInfo g_grad[NLP][NLG][NLG];
MetricInfo g_metric[NLP][NLP];
bool g_cls_ready = false;
// held while a call enqueues its fork / join of the branch streams (the
// events are per device: another thread's record between a fork and its
// waits would redirect them)
std::mutex g_branch_mu;

// side streams and fork / join events of the concurrent (l_a, l_b) branches
int ensure_branches(DevState *ds) {
  if (ds->branches) return DF3C_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (ds->branches) return DF3C_OK;
  for (int b = 0; b < NBRANCH - 1; ++b)
    if (hipStreamCreateWithFlags(&ds->side[b], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ds->join[b], hipEventDisableTiming) != hipSuccess)
      return DF3C_E_HIP;
  if (hipEventCreateWithFlags(&ds->fork, hipEventDisableTiming) != hipSuccess) return DF3C_E_HIP;
  ds->branches = true;
  return DF3C_OK;
}

}  // namespace

// Boys table of device.hpp, F_m(i * BOYS_DT) for m < BOYS_MTAB, row-major
// (generated at build time from the all-positive series in 40-digit decimal
// arithmetic): part of the library's code object, nothing is allocated.  It
// is an ordinary (non-const, external) device variable: a const one has
// internal linkage and, read by no device code of this unit, is left out of
// the code object, where the runtime then cannot find it by name.
__device__ double g_boys_table[BOYS_NGRID * BOYS_MTAB] = {
#include "gen/boys_table.inc"
};

// Workspace of df3c_coulomb_J_noalloc: one copy per device, held until the
// process ends.  In host code this name stands for the device array and is no
// device address: init_device looks up each device's address once (with that
// device current) and only that address is passed to kernels.
static __device__ __align__(256) char scratch[DF3C_NOALLOC_SCRATCH_BYTES];

namespace {

// Host readback slots (pinned, a few ints each): a call that reads counts or
// status words back takes a slot of its own for the duration of the readback,
// so concurrent calls on other streams or threads never share one.
struct PinnedSlots {
  std::mutex mu;
  std::vector<int *> free_slots;
};
PinnedSlots g_slots;
constexpr int SLOT_INTS = 256;  // the largest readback: the NCLS class counts
static_assert(NCLS <= SLOT_INTS, "readback slot smaller than the class counts");

struct Slot {
  int *p = nullptr;
  Slot() {
    {
      std::lock_guard<std::mutex> lk(g_slots.mu);
      if (!g_slots.free_slots.empty()) {
        p = g_slots.free_slots.back();
        g_slots.free_slots.pop_back();
        return;
      }
    }
    if (hipHostMalloc((void **)&p, sizeof(int) * SLOT_INTS) != hipSuccess) p = nullptr;
  }
  ~Slot() {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_slots.mu);
    g_slots.free_slots.push_back(p);
  }
  Slot(const Slot &) = delete;
  Slot &operator=(const Slot &) = delete;
};

// copy n bytes of device memory back through a slot of its own (synchronises s)
hipError_t read_back(void *host, const void *dev, size_t n, hipStream_t s) {
  Slot sl;
  if (!sl.p || n > sizeof(int) * SLOT_INTS) return hipErrorOutOfMemory;
  hipError_t e = hipMemcpyAsync(sl.p, dev, n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) std::memcpy(host, sl.p, n);
  return e;
}

// status of a call from its device word: without DF3C_ASYNC the call reads
// it back (one synchronisation at the end); with it, the word stays in the
// workspace for df3c_workspace_status
int status_of(int word) {
  if (word & 16) return DF3C_E_NUMERIC;  // the fitting solve's pivot test
  if (word & ~2) return DF3C_E_ARG;      // bad index (1), descriptor (4), plan (8)
  return word ? DF3C_E_UNSUPPORTED : DF3C_OK;  // l beyond the build (2)
}
int finish_call(uint32_t flags, const int *err, hipStream_t s) {
  if (flags & DF3C_ASYNC) return DF3C_OK;
  int word = 0;
  if (read_back(&word, err, sizeof(int), s) != hipSuccess) return DF3C_E_HIP;
  return status_of(word);
}

void register_all() {
  if (g_cls_ready) return;
  ClassInfo (*t)[NLA][NLA] = g_cls;
  register_lp0(t[0]);
  register_lp1(t[1]);
  register_lp2(t[2]);
  register_lp3(t[3]);
  register_lp4(t[4]);
  register_lp5(t[5]);
  register_lp6(t[6]);
  register_cart_lp2(t[2]);
  register_cart_lp3(t[3]);
  register_cart_lp4(t[4]);
  register_cart_lp5(t[5]);
  register_cart_lp6(t[6]);
  register_metric_lp0(g_metric[0]);
  register_metric_lp1(g_metric[1]);
  register_metric_lp2(g_metric[2]);
  register_metric_lp3(g_metric[3]);
  register_metric_lp4(g_metric[4]);
  register_metric_lp5(g_metric[5]);
  register_metric_lp6(g_metric[6]);
  register_grad_lp0(g_grad[0]);
  register_grad_lp1(g_grad[1]);
  register_grad_lp2(g_grad[2]);
  register_grad_lp3(g_grad[3]);
  register_grad_lp4(g_grad[4]);
  register_grad_lp5(g_grad[5]);
  register_grad_lp6(g_grad[6]);
  g_cls_ready = true;
}

int init_device(DevState **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return DF3C_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  register_all();
  DevState &s = g_dev[dev];
  if (!s.ready) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_boys_table)) != hipSuccess || !p) return DF3C_E_HIP;
    s.boys = static_cast<const double *>(p);
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return DF3C_E_HIP;
    s.scratch = static_cast<char *>(q);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DF3C_E_HIP;
    s.ncu = prop.multiProcessorCount;
    s.ready = true;
  }
  *out = &s;
  return DF3C_OK;
}

ShellsDev dev_shells(const df3c_shells *b) {
  return ShellsDev{b->nprim, b->prim_off, b->atom, b->exps, b->coefs};
}

bool shells_ok(const df3c_shells *b) {
  return b && b->nshell >= 0 &&
         (b->nshell == 0 || (b->l_host && b->l && b->nprim && b->prim_off && b->atom &&
                             b->exps && b->coefs));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------- launch timing
// When enabled, every class-kernel launch outside graph capture is bracketed by
// a pair of HIP events recorded on its stream; df3c_timing_read returns the
// durations.  Events are pooled and reused across reads.
struct TimedLaunch {
  int kind, cls, dev;
  hipEvent_t e0, e1;
};
bool g_timing = false;
std::vector<TimedLaunch> g_tl;
size_t g_tl_used = 0;

// set while df3c_coulomb_J_noalloc runs on this thread: its launches are not
// timed (the event records could create events and grow the record list)
thread_local bool t_no_alloc = false;

template <class F>
hipError_t timed(int kind, int cls, hipStream_t s, F &&launch) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (!g_timing || t_no_alloc || hipStreamIsCapturing(s, &cap) != hipSuccess ||
      cap != hipStreamCaptureStatusNone)
    return launch();
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_tl_used == g_tl.size()) g_tl.push_back(TimedLaunch{0, 0, -1, nullptr, nullptr});
  TimedLaunch &t = g_tl[g_tl_used];
  if (t.dev != dev) {
    if (t.e0) (void)hipEventDestroy(t.e0);
    if (t.e1) (void)hipEventDestroy(t.e1);
    t.e0 = t.e1 = nullptr;
    if ((e = hipEventCreate(&t.e0)) != hipSuccess || (e = hipEventCreate(&t.e1)) != hipSuccess)
      return e;
    t.dev = dev;
  }
  t.kind = kind;
  t.cls = cls;
  if ((e = hipEventRecord(t.e0, s)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(t.e1, s)) != hipSuccess) return e;
  ++g_tl_used;
  return hipSuccess;
}

// ------------------------------------------------------------ small kernels
__global__ void k_fill_i32(int *p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_zero_f64(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// shell descriptors: contraction degree and centre index in range
// (atom indices in [base, base + natom): a molecule's atoms within a batch)
__global__ void k_check_shells(const int32_t *nprim, const int64_t *prim_off, const int32_t *atom,
                               int32_t n, int32_t natom, int32_t base, int *err) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x)
    if (nprim[s] < 1 || nprim[s] > DF3C_KMAX || prim_off[s] < 0 || atom[s] < base ||
        atom[s] - base >= natom)
      atomicOr(err, 4);
}

void check_shells(const df3c_shells *b, int natom, int *err, hipStream_t s, int base = 0) {
  if (b->nshell <= 0) return;
  const int g = std::min((b->nshell + 255) / 256, 1024);
  hipLaunchKernelGGL(k_check_shells, dim3(g), dim3(256), 0, s, b->nprim, b->prim_off, b->atom,
                     b->nshell, natom, base, err);
}

// class of every triplet; hist[NCLS] counts (aggregated per workgroup in LDS),
// err[0] flags bad input
__global__ void k_classify(const int32_t *trip, int64_t ntrip, const int32_t *laux, int32_t naux,
                           const int32_t *lorb, int32_t norb, uint8_t *cls,
                           int *hist, int *err) {
  __shared__ int h[NCLS];
  for (int i = threadIdx.x; i < NCLS; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < ntrip;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int P = trip[3 * t], a = trip[3 * t + 1], b = trip[3 * t + 2];
    if (P < 0 || P >= naux || a < 0 || a >= norb || b < 0 || b >= norb) {
      atomicOr(err, 1);
      cls[t] = 255;
      continue;
    }
    const int lp = laux[P], la = lorb[a], lb = lorb[b];
    if (lp < 0 || lp > DF3C_LMAX_AUX || la < 0 || la > DF3C_LMAX_ORB || lb < 0 ||
        lb > DF3C_LMAX_ORB) {
      atomicOr(err, 2);
      cls[t] = 255;
      continue;
    }
    const int hi = la >= lb ? la : lb, lo = la >= lb ? lb : la;
    const int c = (lp * NLA + hi) * NLA + lo;
    cls[t] = uint8_t(c);
    atomicAdd(&h[c], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NCLS; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// exclusive scan of hist into cursor (one thread; NCLS is small); start keeps
// the class starts (the scatter advances cursor to the class ends)
__global__ void k_scan(const int *hist, int *cursor, int *start) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int s = 0;
    for (int c = 0; c < NCLS; ++c) {
      cursor[c] = s;
      if (start) start[c] = s;
      s += hist[c];
    }
  }
}

// HRR direction.  Eq. hrr moves quanta from the centre on which VRR1 built
// them (A) to the other one (B) with powers of AB; the transfer is well
// conditioned when the Gaussian product centre P lies near A, i.e. when A's
// exponents dominate.  For equal l the triplet is oriented so that the shell
// with the larger (max exponent x min exponent) carries the VRR1 quanta; for
// unequal l the quanta always go to the lower-l shell (fewest transfers).
__device__ __forceinline__ double shell_tightness(const ShellsDev &b, int s) {
  const int K = b.nprim[s];
  const double *e = b.exps + b.prim_off[s];
  double lo = e[0], hi = e[0];
  for (int i = 1; i < K; ++i) {
    lo = fmin(lo, e[i]);
    hi = fmax(hi, e[i]);
  }
  return lo * hi;
}

__global__ void k_scatter(const int32_t *trip, int64_t ntrip, const int32_t *lorb, ShellsDev orb,
                          const uint8_t *cls, int *cursor, uint32_t *bucket, const int *err) {
  if (*err) return;
  // per round of blockDim.x triplets: rank inside the workgroup from LDS
  // atomics, one global reservation per class and workgroup
  __shared__ int h[NCLS], base[NCLS];
  for (int64_t t0 = blockIdx.x * int64_t(blockDim.x); t0 < ntrip;
       t0 += int64_t(gridDim.x) * blockDim.x) {
    for (int i = threadIdx.x; i < NCLS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    const int c = t < ntrip ? cls[t] : 255;
    int rank = 0;
    uint32_t code = 0;
    if (c != 255) {
      const int a = trip[3 * t + 1], b = trip[3 * t + 2];
      const int la = lorb[a], lb = lorb[b];
      const bool swp =
          la < lb || (la == lb && shell_tightness(orb, b) > shell_tightness(orb, a));
      code = uint32_t(t) | (swp ? 0x80000000u : 0u);
      rank = atomicAdd(&h[c], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NCLS; i += blockDim.x)
      if (h[i]) base[i] = atomicAdd(&cursor[i], h[i]);
    __syncthreads();
    if (c != 255) bucket[base[c] + rank] = code;
    __syncthreads();
  }
}

// grad[x] = sum over team partials, in a fixed order (bitwise reproducible)
__global__ void k_reduce_partial(const double *partial, int nslot, int n, double *grad) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nslot; ++k) s += partial[int64_t(k) * n + x];
    grad[x] = s;
  }
}

// Lanes per shell pair of the register J engine.  It gives one lane to a pair
// and runs every aux shell of the class in that lane, so a class of few pairs
// leaves the SIMDs close to idle; the aux shells are then split between nsub
// lanes of a pair (a power of two <= 16, no more than the aux shells) until
// about four waves per SIMD are resident.
int reg_split(const ClassInfo &ci, int64_t items, int np, int ncu) {
  if (!ci.jreg) return 1;
  const int64_t target = int64_t(ncu) * 4 * 4 * 64;
  int n = 1;
  while (n < 16 && 2 * n <= np && items * n < target) n *= 2;
  return n;
}

int grid_for(int64_t items, int tpw, int ncu) {
  const int64_t need = (items + tpw - 1) / tpw;
  const int64_t cap = int64_t(ncu) * 64;
  return int(std::max<int64_t>(1, std::min(need, cap)));
}

}  // namespace
}  // namespace df3c

using namespace df3c;

extern "C" {

int df3c_init(void) {
  DevState *s = nullptr;
  return init_device(&s);
}

int df3c_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing = on != 0;
  return DF3C_OK;
}

int64_t df3c_timing_read(int32_t *kind, int32_t *cls, float *ms, int64_t cap) {
  if (cap < 0 || (cap > 0 && (!kind || !cls || !ms))) return DF3C_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t n = int64_t(g_tl_used);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return DF3C_E_HIP;
  int rc = DF3C_OK;
  for (int64_t i = 0; i < n && i < cap; ++i) {
    const TimedLaunch &t = g_tl[size_t(i)];
    if (t.dev != cur && hipSetDevice(t.dev) != hipSuccess) { rc = DF3C_E_HIP; break; }
    float v = 0.f;
    if (hipEventSynchronize(t.e1) != hipSuccess || hipEventElapsedTime(&v, t.e0, t.e1) != hipSuccess) {
      rc = DF3C_E_HIP;
      break;
    }
    kind[i] = t.kind;
    cls[i] = t.cls;
    ms[i] = v;
  }
  g_tl_used = 0;
  if (hipSetDevice(cur) != hipSuccess) return DF3C_E_HIP;
  return rc ? rc : n;
}

int df3c_workspace_status(const void *ws, void *stream) {
  if (!ws) return DF3C_E_ARG;
  int word = 0;
  if (read_back(&word, ws, sizeof(int), reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return DF3C_E_HIP;
  return status_of(word);
}

const char *df3c_status_string(int status) {
  switch (status) {
    case DF3C_OK: return "ok";
    case DF3C_E_ARG: return "invalid argument";
    case DF3C_E_UNSUPPORTED: return "unsupported angular momentum or option";
    case DF3C_E_WORKSPACE: return "workspace missing or too small";
    case DF3C_E_HIP: return "HIP runtime error";
    case DF3C_E_NUMERIC: return "matrix not positive definite in working precision";
    default: return "unknown status";
  }
}

size_t df3c_eval_batch_workspace(int64_t ntrip) {
  if (ntrip < 0) ntrip = 0;
  return align256(sizeof(int) * 8) + align256(sizeof(int) * 3 * NCLS) + align256(size_t(ntrip)) +
         align256(sizeof(uint32_t) * size_t(ntrip));
}

int df3c_eval_batch(const double *xyz, int32_t natom, const df3c_shells *aux,
                    const df3c_shells *orb, int64_t ntrip, const int32_t *trip,
                    const int64_t *out_off, double *out, void *ws, size_t ws_bytes, uint32_t flags,
                    void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (ntrip < 0 || ntrip > 0x7fffffff) return DF3C_E_ARG;
  if (ntrip == 0) return DF3C_OK;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !trip || !out_off || !out)
    return DF3C_E_ARG;
  if (orb->pure != 0 || (aux->pure != 0 && aux->pure != 1)) return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_eval_batch_workspace(ntrip)) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(ws);
  int *err = reinterpret_cast<int *>(w);
  w += align256(sizeof(int) * 8);
  int *hist = reinterpret_cast<int *>(w);
  int *cursor = hist + NCLS, *start = hist + 2 * NCLS;
  w += align256(sizeof(int) * 3 * NCLS);
  uint8_t *cls = reinterpret_cast<uint8_t *>(w);
  w += align256(size_t(ntrip));
  uint32_t *bucket = reinterpret_cast<uint32_t *>(w);

  const int g = int(std::min<int64_t>((ntrip + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, err, 8, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, hist, 3 * NCLS, 0);
  check_shells(aux, natom, err, s);
  check_shells(orb, natom, err, s);
  hipLaunchKernelGGL(k_classify, dim3(g), dim3(256), 0, s, trip, ntrip, aux->l, aux->nshell,
                     orb->l, orb->nshell, cls, hist, err);
  StoreArgs a{};
  a.boys = ds->boys;
  a.xyz = xyz;
  a.aux = dev_shells(aux);
  a.orb = dev_shells(orb);
  a.trip = trip;
  a.out_off = out_off;
  a.out = out;
  a.pure = aux->pure;
  a.err = err;
  if (flags & DF3C_ASYNC) {
    // no readback: the scatter and every class kernel read the device status
    // word and the class counts (k_scatter skips a failed batch), so every
    // class the batch could hold is launched; the empty ones exit at once
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, s, hist, cursor, start);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, trip, ntrip, orb->l, dev_shells(orb),
                       cls, cursor, bucket, err);
    for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
      for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
        for (int lb = 0; lb <= la; ++lb) {
          const int c = (lp * NLA + la) * NLA + lb;
          a.bucket = bucket;
          a.dcount = hist + c;
          a.dstart = start + c;
          a.count = ntrip;
          // a Cartesian aux shell of l >= 2 adds the terms of degree l - 2, l - 4, ...
          for (int cs = 0; cs <= (aux->pure ? 0 : lp / 2); ++cs) {
            const ClassInfo &ci = g_cls[lp - 2 * cs][la][lb];
            a.cexp = cs;
            const int grid = std::min(grid_for(ntrip, ci.tpw, ds->ncu), 8 * ds->ncu);
            auto fn = aux->pure ? ci.store : ci.store_cart;
            if (timed(DF3C_KERNEL_STORE, c, s, [&] { return fn(a, grid, s); }) != hipSuccess)
              return DF3C_E_HIP;
          }
        }
    return DF3C_OK;
  }
  // one readback of the class counts and the status word sizes the launches;
  // nothing that dereferences shell data runs before the descriptors are checked
  int rb[NCLS + 8];
  if (read_back(rb, hist, sizeof(int) * NCLS, s) != hipSuccess ||
      read_back(rb + NCLS, err, sizeof(int), s) != hipSuccess)
    return DF3C_E_HIP;
  if (rb[NCLS] & 5) return DF3C_E_ARG;
  if (rb[NCLS] & 2) return DF3C_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, s, hist, cursor, nullptr);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, trip, ntrip, orb->l, dev_shells(orb),
                     cls, cursor, bucket, err);
  // The classes of a batch write disjoint blocks: a batch of several classes
  // runs them on NBRANCH concurrent streams forked from and joined back to s
  // (largest first by triplets x block size; the launches of one class, its
  // Cartesian lower-degree terms included, stay in order on one branch).
  int present = 0;
  for (int c = 0; c < NCLS; ++c) present += rb[c] ? 1 : 0;
  const bool branched = present > 1;
  int branch_of[NCLS] = {};
  std::unique_lock<std::mutex> branch_lock(g_branch_mu, std::defer_lock);
  if (branched) {
    if ((rc = ensure_branches(ds))) return rc;
    branch_lock.lock();
    double cost[NCLS] = {}, load[NBRANCH] = {};
    int cid[NCLS];
    for (int c = 0; c < NCLS; ++c) {
      const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
      cost[c] = double(rb[c]) * (lp + 1) * (lp + 2) * (la + 1) * (la + 2) * (lb + 1) * (lb + 2);
      cid[c] = c;
    }
    std::stable_sort(cid, cid + NCLS, [&](int x, int y) { return cost[x] > cost[y]; });
    for (int k = 0; k < NCLS; ++k) {
      int bmin = 0;
      for (int b = 1; b < NBRANCH; ++b)
        if (load[b] < load[bmin]) bmin = b;
      branch_of[cid[k]] = bmin;
      load[bmin] += cost[cid[k]];
    }
    if (hipEventRecord(ds->fork, s) != hipSuccess) return DF3C_E_HIP;
    for (int b = 0; b < NBRANCH - 1; ++b)
      if (hipStreamWaitEvent(ds->side[b], ds->fork, 0) != hipSuccess) return DF3C_E_HIP;
  }
  int64_t off = 0;
  int brc = DF3C_OK;
  for (int c = 0; c < NCLS && !brc; ++c) {
    if (!rb[c]) continue;
    const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
    hipStream_t bs = (!branched || branch_of[c] == 0) ? s : ds->side[branch_of[c] - 1];
    a.bucket = bucket + off;
    a.count = rb[c];
    // a Cartesian aux shell of l >= 2: the launches of classes l - 2, l - 4, ...
    // add the lower-degree terms of its expansion into the same blocks
    for (int cs = 0; cs <= (aux->pure ? 0 : lp / 2) && !brc; ++cs) {
      const ClassInfo &ci = g_cls[lp - 2 * cs][la][lb];
      a.cexp = cs;
      auto fn = aux->pure ? ci.store : ci.store_cart;
      if (timed(DF3C_KERNEL_STORE, c, bs,
                [&] { return fn(a, grid_for(rb[c], ci.tpw, ds->ncu), bs); }) != hipSuccess)
        brc = DF3C_E_HIP;
    }
    off += rb[c];
  }
  if (branched)
    for (int b = 0; b < NBRANCH - 1; ++b)
      if (hipEventRecord(ds->join[b], ds->side[b]) != hipSuccess ||
          hipStreamWaitEvent(s, ds->join[b], 0) != hipSuccess)
        return DF3C_E_HIP;
  return brc;
}

// ------------------------------------------------------------------- DF-J
namespace {
// ------------------------------------------------------------ device plans
// The shell lists of a single-molecule call are built on the device from the
// shells' own l and nprim (no host-built plan is uploaded, so the calls that
// use them are asynchronous and can be captured in a HIP graph).  One
// workgroup of PLAN_TPB threads per basis:
//   sorted[]  shells grouped by key, ascending, stable in shell order; the
//             orbital key is l * 64 + 63 - min(nprim, 63) (decreasing
//             contraction degree within l: the shell pairs that share a
//             wavefront then run equal primitive loops), the aux key is l;
//   off[]     function offset of every shell in shell order (off[n] = total):
//             ncart(l) functions per orbital shell, npure or ncart per aux
//             shell;
//   pmap[]    optional (solid-harmonic orbital shells): pmap[po[s] + m] =
//             s << 4 | m over the 2l+1 functions of each shell, po the pure
//             offsets;
//   cmap[]    optional: cmap[off[s] + i] = s << 4 | i over the Cartesian
//             components, with the pure offsets in poff[];
// and the number of shells of each l is compared with the host's count (the
// launches are sized from l_host): a mismatch or an l beyond the build sets
// bit 8 of *err.
constexpr int PLAN_TPB = 1024;
constexpr int PLAN_WAVES = PLAN_TPB / 64;
constexpr int PLAN_NKEY = (DF3C_LMAX_AUX + 1) * 64;
struct PlanCounts {
  int32_t n[DF3C_LMAX_AUX + 1];
};

__device__ __forceinline__ int plan_key(int l, int k, bool orb) {
  return orb ? l * 64 + 63 - min(max(k, 1), 63) : l * 64;
}

__global__ void __launch_bounds__(PLAN_TPB)
    k_plan_shells(const int32_t *l, const int32_t *nprim, int32_t n, int32_t lmax, int32_t orb,
                  int32_t pure, PlanCounts hc, int32_t *sorted, int64_t *off, int32_t *pmap,
                  int32_t *cmap, int64_t *poff, int *err) {
  __shared__ int hist[PLAN_WAVES][PLAN_NKEY];  // per-wave counts, then running bases
  __shared__ int kstart[PLAN_NKEY];
  __shared__ int64_t wsum[PLAN_WAVES][2];
  __shared__ int bad;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < PLAN_WAVES * PLAN_NKEY; i += PLAN_TPB) (&hist[0][0])[i] = 0;
  if (tid == 0) bad = 0;
  __syncthreads();
  // each wave owns a contiguous slice of the shells
  const int per = (n + PLAN_WAVES - 1) / PLAN_WAVES;
  const int s0 = min(n, w * per), s1 = min(n, s0 + per);
  auto keyof = [&](int s) {
    const int ls = l[s];
    if (ls < 0 || ls > lmax) {
      bad = 1;
      return 0;
    }
    return plan_key(ls, orb ? nprim[s] : 1, orb != 0);
  };
  for (int s = s0 + lane; s < s1; s += 64) atomicAdd(&hist[w][keyof(s)], 1);
  __syncthreads();
  // key totals -> exclusive key starts (log-step scan); per-wave bases
  int tot = 0;
  if (tid < PLAN_NKEY) {
    for (int v = 0; v < PLAN_WAVES; ++v) {
      const int c = hist[v][tid];
      hist[v][tid] = tot;
      tot += c;
    }
    kstart[tid] = tot;
  }
  __syncthreads();
  for (int o = 1; o < PLAN_NKEY; o <<= 1) {
    const int v = (tid < PLAN_NKEY && tid >= o) ? kstart[tid - o] : 0;
    __syncthreads();
    if (tid < PLAN_NKEY) kstart[tid] += v;
    __syncthreads();
  }
  if (tid < PLAN_NKEY) kstart[tid] -= tot;  // inclusive -> exclusive
  __syncthreads();
  // shells per l against the host's counts
  if (tid <= DF3C_LMAX_AUX) {
    const int hi = tid == DF3C_LMAX_AUX ? 0 : kstart[(tid + 1) * 64];
    const int cnt = (tid == DF3C_LMAX_AUX ? n : hi) - kstart[tid * 64];
    const int want = tid <= lmax ? hc.n[tid] : 0;
    if (cnt != want) bad = 1;
  }
  // stable scatter: every wave walks its slice in order, 64 shells at a time;
  // the lanes of one key are ranked by a ballot
  for (int c0 = s0; c0 < s1; c0 += 64) {
    const int s = c0 + lane;
    const bool act = s < s1;
    const int k = act ? keyof(s) : -1;
    unsigned long long rem = __ballot(act);
    while (rem) {
      const int lead = __ffsll(rem) - 1;
      const int lk = __shfl(k, lead);
      const unsigned long long m = __ballot(act && k == lk);
      const int base = kstart[lk] + hist[w][lk];
      if (act && k == lk) sorted[base + __popcll(m & ((1ull << lane) - 1))] = s;
      if (lane == lead) hist[w][lk] += __popcll(m);
      rem &= ~m;
    }
  }
  // offsets in shell order: block-wide scans of the function counts (ncart or
  // npure, and npure for the pure maps), tile by tile
  int64_t carry0 = 0, carry1 = 0;
  if (tid == 0) off[0] = 0;
  if (tid == 0 && poff) poff[0] = 0;
  for (int t0 = 0; t0 < n; t0 += PLAN_TPB) {
    const int s = t0 + tid;
    int ls = s < n ? l[s] : 0;
    ls = min(max(ls, 0), lmax);
    const int nc = (ls + 1) * (ls + 2) / 2, np = 2 * ls + 1;
    int64_t v0 = s < n ? ((orb || !pure) ? nc : np) : 0, v1 = s < n ? np : 0;
    // inclusive scan within the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t a0 = __shfl_up(v0, o), a1 = __shfl_up(v1, o);
      if (lane >= o) {
        v0 += a0;
        v1 += a1;
      }
    }
    if (lane == 63) {
      wsum[w][0] = v0;
      wsum[w][1] = v1;
    }
    __syncthreads();
    int64_t b0 = carry0, b1 = carry1;
    for (int v = 0; v < w; ++v) {
      b0 += wsum[v][0];
      b1 += wsum[v][1];
    }
    if (s < n) {
      off[s + 1] = b0 + v0;
      if (poff) poff[s + 1] = b1 + v1;
      const int64_t f0 = b0 + v0 - ((orb || !pure) ? nc : np), f1 = b1 + v1 - np;
      if (pmap)
        for (int m = 0; m < np; ++m) pmap[f1 + m] = s << 4 | m;
      if (cmap)
        for (int i = 0; i < nc; ++i) cmap[f0 + i] = s << 4 | i;
    }
    for (int v = 0; v < PLAN_WAVES; ++v) {
      carry0 += wsum[v][0];
      carry1 += wsum[v][1];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) atomicOr(err, 8);
}

extern "C++" {
// Host half of a single-molecule plan, from l_host: the shells of every l
// (the class ranges of the sorted lists the device plan fills), their counts
// for the device's check, and the function totals.
struct HostPlan {
  int32_t orb_start[DF3C_LMAX_ORB + 2] = {}, aux_start[DF3C_LMAX_AUX + 2] = {};
  PlanCounts co{}, ca{};
  int64_t nao = 0, naux = 0, npure = 0;  // Cartesian AOs, aux functions, pure AOs
};

int host_plan(const df3c_shells *aux, const df3c_shells *orb, HostPlan &p) {
  if ((orb->nshell && !orb->l_host) || (aux->nshell && !aux->l_host)) return DF3C_E_ARG;
  for (int s = 0; s < orb->nshell; ++s) {
    const int l = orb->l_host[s];
    if (l < 0 || l > DF3C_LMAX_ORB) return DF3C_E_UNSUPPORTED;
    p.co.n[l]++;
    p.nao += (l + 1) * (l + 2) / 2;
    p.npure += 2 * l + 1;
  }
  for (int s = 0; s < aux->nshell; ++s) {
    const int l = aux->l_host[s];
    if (l < 0 || l > DF3C_LMAX_AUX) return DF3C_E_UNSUPPORTED;
    if (!aux->pure && l > 1) return DF3C_E_UNSUPPORTED;
    p.ca.n[l]++;
    p.naux += aux->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2;
  }
  for (int l = 0; l <= DF3C_LMAX_ORB; ++l) p.orb_start[l + 1] = p.orb_start[l] + p.co.n[l];
  for (int l = 0; l <= DF3C_LMAX_AUX; ++l) p.aux_start[l + 1] = p.aux_start[l] + p.ca.n[l];
  return DF3C_OK;
}

// Device half, at the start of the workspace: status word, sorted shell
// lists, function offsets, aux-shell records.
struct DevPlan {
  int *err = nullptr;
  int32_t *orb_sorted = nullptr, *aux_sorted = nullptr;
  int64_t *ao_off = nullptr, *aux_off = nullptr;
  double *arec = nullptr;
};

size_t jplan_bytes(int64_t norb, int64_t naux) {
  return align256(sizeof(int) * 8) + align256(sizeof(int32_t) * norb) + align256(sizeof(int32_t) * naux) +
         align256(sizeof(int64_t) * (norb + 1)) + align256(sizeof(int64_t) * (naux + 1)) +
         align256(sizeof(double) * AREC * naux);
}

DevPlan carve_plan(void *ws, int64_t norb, int64_t naux) {
  DevPlan d;
  char *w = static_cast<char *>(ws);
  d.err = reinterpret_cast<int *>(w);
  w += align256(sizeof(int) * 8);
  d.orb_sorted = reinterpret_cast<int32_t *>(w);
  w += align256(sizeof(int32_t) * norb);
  d.aux_sorted = reinterpret_cast<int32_t *>(w);
  w += align256(sizeof(int32_t) * naux);
  d.ao_off = reinterpret_cast<int64_t *>(w);
  w += align256(sizeof(int64_t) * (norb + 1));
  d.aux_off = reinterpret_cast<int64_t *>(w);
  w += align256(sizeof(int64_t) * (naux + 1));
  d.arec = reinterpret_cast<double *>(w);
  return d;
}

// zero the status word, check both bases' descriptors, build both shell
// lists (pmap / cmap + poff: optional maps of a solid-harmonic orbital basis)
hipError_t launch_plan(const DevPlan &d, const HostPlan &hp, const df3c_shells *aux,
                       const df3c_shells *orb, int natom, int32_t *pmap, int32_t *cmap,
                       int64_t *poff, hipStream_t s, int atom_base = 0) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, d.err, 8, 0);
  check_shells(aux, natom, d.err, s, atom_base);
  check_shells(orb, natom, d.err, s, atom_base);
  hipLaunchKernelGGL(k_plan_shells, dim3(1), dim3(PLAN_TPB), 0, s, orb->l, orb->nprim,
                     orb->nshell, DF3C_LMAX_ORB, 1, 0, hp.co, d.orb_sorted, d.ao_off, pmap, cmap,
                     poff, d.err);
  hipLaunchKernelGGL(k_plan_shells, dim3(1), dim3(PLAN_TPB), 0, s, aux->l, aux->nprim,
                     aux->nshell, DF3C_LMAX_AUX, 0, aux->pure, hp.ca, d.aux_sorted, d.aux_off,
                     nullptr, nullptr, nullptr, d.err);
  return hipGetLastError();
}

}  // extern "C++"


extern "C++" {
// d' = T^T d_P of one aux shell of l = LP into its record
template <int LP>
__device__ void aux_dq(const double *dP, int pure, double *dq) {
  constexpr int NCP = ncart(LP);
  if (pure) {
    for (int c = 0; c < NCP; ++c) {
      double v = 0.0;
      for (int m = 0; m < npure(LP); ++m) v += GenSolid<LP>::dense[m * NCP + c] * dP[m];
      dq[c] = v;
    }
  } else {
    for (int c = 0; c < NCP; ++c) dq[c] = dP[c];
  }
}

// aux-shell records of the sorted aux list (d may be null: no d')
__global__ void k_aux_records(const int32_t *sorted, int64_t n, const int32_t *lsh, ShellsDev aux,
                              const double *xyz, const int64_t *aux_off, const double *d,
                              int32_t pure, double *rec, const int *err) {
  if (err && *err) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int s = sorted[i];
    const int at = aux.atom[s];
    double *r = rec + i * AREC;
    r[AR_CX] = xyz[3 * at];
    r[AR_CY] = xyz[3 * at + 1];
    r[AR_CZ] = xyz[3 * at + 2];
    r[AR_PRIM] = double(aux.prim_off[s]);
    r[AR_K] = double(aux.nprim[s]);
    r[AR_ATOM] = double(at);
    const bool has = aux.nprim[s] > 0;
    r[AR_Z0] = has ? aux.exps[aux.prim_off[s]] : 0.0;
    r[AR_C0] = has ? aux.coefs[aux.prim_off[s]] : 0.0;
    if (!d) continue;
    const double *dP = d + aux_off[s];
    switch (lsh[s]) {
      case 0: aux_dq<0>(dP, pure, r + AR_DQ); break;
      case 1: aux_dq<1>(dP, pure, r + AR_DQ); break;
      case 2: aux_dq<2>(dP, pure, r + AR_DQ); break;
      case 3: aux_dq<3>(dP, pure, r + AR_DQ); break;
      case 4: aux_dq<4>(dP, pure, r + AR_DQ); break;
      case 5: aux_dq<5>(dP, pure, r + AR_DQ); break;
      default: aux_dq<6>(dP, pure, r + AR_DQ); break;
    }
  }
}
}  // extern "C++"

hipError_t launch_aux_records(const int32_t *sorted, int64_t n, const df3c_shells *aux,
                              const double *xyz, const int64_t *aux_off, const double *d,
                              double *rec, hipStream_t s, const int *err = nullptr) {
  if (n <= 0) return hipSuccess;
  const int grid = int(std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(k_aux_records, dim3(grid), dim3(256), 0, s, sorted, n, aux->l,
                     dev_shells(aux), xyz, aux_off, d, aux->pure, rec, err);
  return hipGetLastError();
}
}  // namespace

namespace {
// workspace of the solid-harmonic orbital transform (pure-row map, Cartesian J)
size_t pure_bytes(const df3c_shells *orb) {
  if (!orb->pure) return 0;
  int64_t nc = 0, np = 0;
  for (int s = 0; s < orb->nshell; ++s) {
    const int l = std::min(std::max(orb->l_host[s], 0), DF3C_LMAX_ORB);
    nc += (l + 1) * (l + 2) / 2;
    np += 2 * l + 1;
  }
  return align256(sizeof(int32_t) * np) + align256(sizeof(double) * nc * nc);
}
// pull-back of a matrix over pure orbital functions to the Cartesian blocks
// (gradient G, gamma D): Cartesian-row map, pure shell offsets, the result
size_t pullback_bytes(const df3c_shells *orb) {
  if (!orb->pure) return 0;
  int64_t nc = 0;
  for (int s = 0; s < orb->nshell; ++s) {
    const int l = std::min(std::max(orb->l_host[s], 0), DF3C_LMAX_ORB);
    nc += (l + 1) * (l + 2) / 2;
  }
  return align256(sizeof(int32_t) * nc) + align256(sizeof(int64_t) * (orb->nshell + 1)) +
         align256(sizeof(double) * nc * nc);
}
}  // namespace

size_t df3c_coulomb_J_workspace(const df3c_shells *aux, const df3c_shells *orb) {
  if (!shells_ok(aux) || !shells_ok(orb)) return 0;
  return jplan_bytes(orb->nshell, aux->nshell) + pure_bytes(orb);
}

namespace {
// shell-pair screening: S_ab = max_ij |c c'| (pi/(z+z'))^{3/2} exp(-z z'/(z+z') AB^2)
__global__ void k_screen_pairs(const double *xyz, ShellsDev orb, int32_t n, double tau,
                               uint8_t *mask) {
  const int64_t total = int64_t(n) * n;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int sa = int(x / n), sb = int(x - int64_t(sa) * n);
    const int ia = orb.atom[sa], ib = orb.atom[sb];
    const double dx = xyz[3 * ia] - xyz[3 * ib], dy = xyz[3 * ia + 1] - xyz[3 * ib + 1],
                 dz = xyz[3 * ia + 2] - xyz[3 * ib + 2];
    const double ab2 = dx * dx + dy * dy + dz * dz;
    const double *ea = orb.exps + orb.prim_off[sa], *ca = orb.coefs + orb.prim_off[sa];
    const double *eb = orb.exps + orb.prim_off[sb], *cb = orb.coefs + orb.prim_off[sb];
    double smax = 0.0;
    for (int i = 0; i < orb.nprim[sa]; ++i)
      for (int j = 0; j < orb.nprim[sb]; ++j) {
        const double g = ea[i] + eb[j], t = 3.14159265358979323846 / g;
        smax = fmax(smax, fabs(ca[i] * cb[j]) * t * sqrt(t) * exp(-ea[i] * eb[j] / g * ab2));
      }
    mask[x] = smax >= tau ? 1 : 0;
  }
}

// indices q of a class's pairs (as the kernels decode them) that the mask
// keeps, in increasing q.  One workgroup per (l_a, l_b) class, all classes in
// one launch: thread t scans a contiguous range of q, the ranges' counts are
// scanned in LDS (log-step scan of integers), then every thread writes its
// kept indices in order (deterministic; an all-ones mask gives q = 0, 1, ...)
constexpr int COMPACT_TPB = 1024;
constexpr int NCOMPACT = NLA * (NLA + 1) / 2;  // (l_a >= l_b) classes
struct CompactJob {
  const int32_t *ash, *bsh;
  int32_t nb, same;
  int64_t npair;
  int64_t *plist;
  unsigned long long *count;
};
struct CompactJobs {
  CompactJob j[NCOMPACT];
};
__global__ void __launch_bounds__(COMPACT_TPB)
    k_pair_compact(CompactJobs jobs, const uint8_t *mask, int32_t nshell, const int *err) {
  __shared__ int64_t cnt[COMPACT_TPB];
  if (*err) return;
  const CompactJob &job = jobs.j[blockIdx.x];
  const int32_t *ash = job.ash, *bsh = job.bsh;
  const int32_t nb = job.nb, same = job.same;
  const int64_t npair = job.npair;
  const int t = threadIdx.x;
  const int64_t per = (npair + COMPACT_TPB - 1) / COMPACT_TPB;
  const int64_t q0 = std::min<int64_t>(npair, int64_t(t) * per);
  const int64_t q1 = std::min<int64_t>(npair, q0 + per);
  auto kept = [&](int64_t q) {
    int sa, sb;
    if (same) {
      int i = int((sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
      while (int64_t(i) * (i + 1) / 2 > q) --i;
      while (int64_t(i + 1) * (i + 2) / 2 <= q) ++i;
      sa = ash[i];
      sb = ash[int(q - int64_t(i) * (i + 1) / 2)];
    } else {
      const int i = int(q / nb);
      sa = ash[i];
      sb = bsh[int(q - int64_t(i) * nb)];
    }
    return mask[int64_t(sa) * nshell + sb] != 0;
  };
  int64_t c = 0;
  for (int64_t q = q0; q < q1; ++q) c += kept(q) ? 1 : 0;
  cnt[t] = c;
  __syncthreads();
  for (int off = 1; off < COMPACT_TPB; off <<= 1) {  // inclusive scan
    const int64_t v = t >= off ? cnt[t - off] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  if (t == COMPACT_TPB - 1) *job.count = (unsigned long long)cnt[t];
  int64_t o = cnt[t] - c;
  for (int64_t q = q0; q < q1; ++q)
    if (kept(q)) job.plist[o++] = q;
}

// shell pairs of all (l_a >= l_b) classes (the masked J's pair lists)
int64_t total_class_pairs(const df3c_shells *orb) {
  int64_t n[DF3C_LMAX_ORB + 1] = {};
  for (int s = 0; s < orb->nshell; ++s)
    if (orb->l_host[s] >= 0 && orb->l_host[s] <= DF3C_LMAX_ORB) ++n[orb->l_host[s]];
  int64_t m = 1;
  for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
    for (int lb = 0; lb <= la; ++lb) m += la == lb ? n[la] * (n[la] + 1) / 2 : n[la] * n[lb];
  return m;
}

// Solid-harmonic orbital shells: J is built over the Cartesian components
// and each block is transformed on both sides afterwards (the solid-harmonic
// transform is linear per shell, Section 2.5.1), from the sparse rows of the
// same real solid-harmonic table as the ket.  Workspace past the J plan: the
// pure-row map (shell << 4 | m) and the Cartesian J.
extern "C++" {
template <int L>
__device__ inline void solid_row(int m, int &n, const int16_t *&col, const double *&val) {
  const int b = GenSolid<L>::start[m];
  n = GenSolid<L>::start[m + 1] - b;
  col = GenSolid<L>::col + b;
  val = GenSolid<L>::val + b;
}

__device__ inline void solid_row_l(int l, int m, int &n, const int16_t *&col, const double *&val) {
  switch (l) {
    case 0: solid_row<0>(m, n, col, val); break;
    case 1: solid_row<1>(m, n, col, val); break;
    case 2: solid_row<2>(m, n, col, val); break;
    case 3: solid_row<3>(m, n, col, val); break;
    default: solid_row<4>(m, n, col, val); break;
  }
}

// dense [2l+1][ncart(l)] rows of the same table
__device__ inline const double *solid_dense_l(int l) {
  switch (l) {
    case 0: return GenSolid<0>::dense;
    case 1: return GenSolid<1>::dense;
    case 2: return GenSolid<2>::dense;
    case 3: return GenSolid<3>::dense;
    default: return GenSolid<4>::dense;
  }
}
}  // extern "C++"

// J[r][c] = sum_ij T_la[m_r][i] T_lb[m_c][j] Jc[cao[sa] + i][cao[sb] + j] for
// the pure rows r, c (one thread per element of J, rows of J contiguous;
// an element above the diagonal is evaluated as its mirror)
__global__ void k_bra_pure(const double *Jc, int64_t nc, const int32_t *pmap,
                           const int64_t *cao, const int32_t *lsh, double *J, int64_t np,
                           const int *err) {
  if (*err) return;
  const int64_t total = np * np;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    // both triangles from the same arithmetic (Jc is exactly symmetric)
    int64_t r = x / np, c = x - r * np;
    if (r < c) {
      const int64_t t = r;
      r = c;
      c = t;
    }
    const int sa = pmap[r] >> 4, ma = pmap[r] & 15, sb = pmap[c] >> 4, mb = pmap[c] & 15;
    int na, nb;
    const int16_t *ca, *cb;
    const double *va, *vb;
    solid_row_l(lsh[sa], ma, na, ca, va);
    solid_row_l(lsh[sb], mb, nb, cb, vb);
    const double *row = Jc + cao[sa] * nc + cao[sb];
    double v = 0.0;
    for (int i = 0; i < na; ++i) {
      double t = 0.0;
      for (int j = 0; j < nb; ++j) t += vb[j] * row[int64_t(ca[i]) * nc + cb[j]];
      v += va[i] * t;
    }
    J[x] = v;
  }
}

// Gradient with solid-harmonic orbital shells: L = sum G_pure J_pure equals
// sum G_cart J_cart with G_cart = T_a^T G_pure T_b per block, so G is pulled
// back once and the Cartesian gradient engines run unchanged.
//   Gc[r][c] = sum_mn T_la[m][i_r] T_lb[n][j_c] G[poff[sa] + m][poff[sb] + n]
__global__ void k_bra_cart(const double *G, int64_t np, const int32_t *cmap,
                           const int64_t *poff, const int32_t *lsh, double *Gc, int64_t nc,
                           const int *err) {
  if (*err) return;
  const int64_t total = nc * nc;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = x / nc, c = x - r * nc;
    const int sa = cmap[r] >> 4, ia = cmap[r] & 15, sb = cmap[c] >> 4, ib = cmap[c] & 15;
    const int la = lsh[sa], lb = lsh[sb];
    const int nca = (la + 1) * (la + 2) / 2, ncb = (lb + 1) * (lb + 2) / 2;
    const double *Ta = solid_dense_l(la), *Tb = solid_dense_l(lb);
    const double *row = G + poff[sa] * np + poff[sb];
    double v = 0.0;
    for (int m = 0; m < 2 * la + 1; ++m) {
      const double ta = Ta[m * nca + ia];
      if (ta == 0.0) continue;
      double t = 0.0;
      for (int n = 0; n < 2 * lb + 1; ++n) t += Tb[n * ncb + ib] * row[int64_t(m) * np + n];
      v += ta * t;
    }
    Gc[x] = v;
  }
}

extern "C++" {
// Pull-back workspace (pullback_bytes(orb) bytes at q): the Cartesian-row
// map and pure shell offsets, which the device plan fills, and Gc.
struct PullBack {
  int32_t *cmap = nullptr;
  int64_t *poff = nullptr;
  double *Gc = nullptr;
};
PullBack carve_pullback(const df3c_shells *orb, char *q, int64_t nc) {
  PullBack p;
  p.cmap = reinterpret_cast<int32_t *>(q);
  q += align256(sizeof(int32_t) * nc);
  p.poff = reinterpret_cast<int64_t *>(q);
  q += align256(sizeof(int64_t) * (orb->nshell + 1));
  p.Gc = reinterpret_cast<double *>(q);
  return p;
}
// Gc = T_a^T G T_b per block (asynchronous)
hipError_t pull_back_cart(const df3c_shells *orb, const double *G, const PullBack &pb, int64_t nc,
                          int64_t np, const int *err, hipStream_t s) {
  if (!nc) return hipSuccess;
  hipLaunchKernelGGL(k_bra_cart, dim3(int(std::min<int64_t>((nc * nc + 255) / 256, 8192))),
                     dim3(256), 0, s, G, np, pb.cmap, pb.poff, orb->l, pb.Gc, nc, err);
  return hipGetLastError();
}
}  // extern "C++"

// DF-J over all pairs (mask null) or over the pairs the mask keeps.  Every
// step is enqueued on s: the plan is built on the device, the status word
// guards every kernel that reads shell data, and no host memory is read
// after the call returns (asynchronous, capturable).  `scratch` is the
// workspace past the plan (masked pair lists, then the pure-orbital maps and
// the Cartesian J).
int coulomb_J_run(const double *xyz, int32_t natom, const df3c_shells *aux,
                  const df3c_shells *orb, const double *d, const uint8_t *mask, double *J,
                  void *ws, uint32_t flags, hipStream_t s) {
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  HostPlan p;
  if ((rc = host_plan(aux, orb, p))) return rc;
  if (orb->pure && orb->nshell >= (1 << 27)) return DF3C_E_UNSUPPORTED;  // rows packed shell << 4
  const DevPlan dp = carve_plan(ws, orb->nshell, aux->nshell);
  char *w = static_cast<char *>(ws) + jplan_bytes(orb->nshell, aux->nshell);
  // masked only: kept-pair counters and lists of the (l_a, l_b) classes
  unsigned long long *pcount = nullptr;
  int64_t *plist = nullptr;
  if (mask) {
    pcount = reinterpret_cast<unsigned long long *>(w);
    plist = reinterpret_cast<int64_t *>(w + align256(sizeof(unsigned long long) * NLA * NLA));
    w += align256(sizeof(unsigned long long) * NLA * NLA) +
         align256(sizeof(int64_t) * size_t(total_class_pairs(orb)));
  }
  // pure orbital shells: the engines fill the Cartesian J in the workspace
  double *Jout = J;
  int32_t *pmap = nullptr;
  if (orb->pure) {
    pmap = reinterpret_cast<int32_t *>(w);
    J = reinterpret_cast<double *>(w + align256(sizeof(int32_t) * p.npure));
  }
  if (launch_plan(dp, p, aux, orb, natom, pmap, nullptr, nullptr, s) != hipSuccess)
    return DF3C_E_HIP;
  const int64_t nJ = p.nao * p.nao;
  hipLaunchKernelGGL(k_zero_f64, dim3(int(std::min<int64_t>((nJ + 255) / 256, 4096))), dim3(256),
                     0, s, J, nJ);
  if (launch_aux_records(dp.aux_sorted, aux->nshell, aux, xyz, dp.aux_off, d, dp.arec, s,
                         dp.err) != hipSuccess)
    return DF3C_E_HIP;
  JArgs a{};
  a.boys = ds->boys;
  a.xyz = xyz;
  a.aux = dev_shells(aux);
  a.orb = dev_shells(orb);
  a.ao_off = dp.ao_off;
  a.aux_off = dp.aux_off;
  a.d = d;
  a.J = J;
  a.nao = p.nao;
  a.pure = aux->pure;
  a.err = dp.err;
  auto launch = [&](int lp, int la, int lb, hipStream_t ls) -> int {
    const int np = p.aux_start[lp + 1] - p.aux_start[lp];
    if (!np) return DF3C_OK;
    a.psh = dp.aux_sorted + p.aux_start[lp];
    a.arec = dp.arec + int64_t(p.aux_start[lp]) * AREC;
    a.np = np;
    const ClassInfo &ci = g_cls[lp][la][lb];
    const int c = (lp * NLA + la) * NLA + lb;
    a.nsub = reg_split(ci, a.npair, a.np, ds->ncu);
    if (timed(DF3C_KERNEL_J, c, ls, [&] {
          return ci.jfn(a, grid_for(a.npair, ci.tpwj / a.nsub, ds->ncu), ls);
        }) != hipSuccess)
      return DF3C_E_HIP;
    return DF3C_OK;
  };
  auto set_class = [&](int la, int lb) {
    const int na = p.orb_start[la + 1] - p.orb_start[la];
    const int nb = p.orb_start[lb + 1] - p.orb_start[lb];
    a.ash = dp.orb_sorted + p.orb_start[la];
    a.bsh = dp.orb_sorted + p.orb_start[lb];
    a.na = na;
    a.nb = nb;
    a.same = (la == lb);
    a.npair = (la == lb) ? int64_t(na) * (na + 1) / 2 : int64_t(na) * nb;
    return na > 0 && nb > 0;
  };
  // Classes of different (l_a, l_b) write disjoint J blocks: the groups run
  // on NBRANCH concurrent streams forked from and joined back to s (also
  // under capture, as parallel graph branches); inside a group the L_P
  // classes keep ascending order, so every J element sums its classes in
  // the same sequence as on one stream.  Groups go to branches longest
  // first by a work model (pairs x aux functions x Cartesian pair size).
  // prep(la, lb) sets the group's arguments up and tells whether it runs.
  auto run_branches = [&](auto prep) -> int {
    int e = ensure_branches(ds);
    if (e) return e;
    std::lock_guard<std::mutex> lk(g_branch_mu);
    double gcost[NLA * NLA] = {}, load[NBRANCH] = {};
    int branch_of[NLA * NLA] = {};
    for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        if (!prep(la, lb)) continue;
        for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
          gcost[la * NLA + lb] += double(a.npair) * double(p.aux_start[lp + 1] - p.aux_start[lp]) *
                                  (2 * lp + 1) * (la + 1) * (la + 2) * (lb + 1) * (lb + 2);
      }
    int gid[NLA * NLA];
    for (int g = 0; g < NLA * NLA; ++g) gid[g] = g;
    std::stable_sort(gid, gid + NLA * NLA, [&](int x, int y) { return gcost[x] > gcost[y]; });
    for (int k = 0; k < NLA * NLA; ++k) {
      int bmin = 0;
      for (int b = 1; b < NBRANCH; ++b)
        if (load[b] < load[bmin]) bmin = b;
      branch_of[gid[k]] = bmin;
      load[bmin] += gcost[gid[k]];
    }
    if (hipEventRecord(ds->fork, s) != hipSuccess) return int(DF3C_E_HIP);
    for (int b = 0; b < NBRANCH - 1; ++b)
      if (hipStreamWaitEvent(ds->side[b], ds->fork, 0) != hipSuccess) return int(DF3C_E_HIP);
    int brc = DF3C_OK;
    for (int la = 0; la <= DF3C_LMAX_ORB && !brc; ++la)
      for (int lb = 0; lb <= la && !brc; ++lb) {
        if (!prep(la, lb)) continue;
        const int br = branch_of[la * NLA + lb];
        hipStream_t bs = br == 0 ? s : ds->side[br - 1];
        for (int lp = 0; lp <= DF3C_LMAX_AUX && !brc; ++lp) brc = launch(lp, la, lb, bs);
      }
    // join every branch back to s, also after a failed launch
    for (int b = 0; b < NBRANCH - 1; ++b)
      if (hipEventRecord(ds->join[b], ds->side[b]) != hipSuccess ||
          hipStreamWaitEvent(s, ds->join[b], 0) != hipSuccess)
        return int(DF3C_E_HIP);
    return brc;
  };
  if (!mask) {
    if ((rc = run_branches(set_class))) return rc;
  } else {
    // masked: the kept pairs of every (l_a, l_b) class are compacted into the
    // class's list on the device; every launch is sized for the whole class
    // and the kernels read the kept count (each J element still sums l_P in
    // ascending order)
    int64_t loff[NLA][NLA] = {};
    int64_t o = 0;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int *>(pcount),
                       2 * NLA * NLA, 0);
    CompactJobs jobs{};
    int nj = 0;
    for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        loff[la][lb] = o;
        if (!set_class(la, lb)) continue;
        jobs.j[nj++] = CompactJob{a.ash, a.bsh, a.nb, a.same, a.npair, plist + o,
                                  pcount + la * NLA + lb};
        o += a.npair;
      }
    if (nj) {
      hipLaunchKernelGGL(k_pair_compact, dim3(nj), dim3(COMPACT_TPB), 0, s, jobs, mask,
                         orb->nshell, dp.err);
      if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
    }
    // without DF3C_ASYNC the kept counts are read back once and size the
    // launches (lanes per pair and grid for the pairs that remain)
    unsigned long long kept[NLA * NLA] = {};
    const bool sized = !(flags & DF3C_ASYNC);
    if (sized && read_back(kept, pcount, sizeof(kept), s) != hipSuccess) return DF3C_E_HIP;
    auto prep = [&](int la, int lb) {
      if (!set_class(la, lb)) return false;
      a.plist = plist + loff[la][lb];
      a.pcount = reinterpret_cast<const int64_t *>(pcount + la * NLA + lb);
      if (sized) a.npair = int64_t(kept[la * NLA + lb]);  // the kernels read *pcount
      return a.npair > 0;
    };
    if ((rc = run_branches(prep))) return rc;
  }
  if (orb->pure && p.npure) {
    const int64_t n2 = p.npure * p.npure;
    hipLaunchKernelGGL(k_bra_pure, dim3(int(std::min<int64_t>((n2 + 255) / 256, 8192))),
                       dim3(256), 0, s, J, p.nao, pmap, dp.ao_off, orb->l, Jout, p.npure, dp.err);
    if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  }
  return finish_call(flags, dp.err, s);
}
}  // namespace

int df3c_coulomb_J(const double *xyz, int32_t natom, const df3c_shells *aux,
                   const df3c_shells *orb, const double *d, double *J, void *ws, size_t ws_bytes,
                   uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !J) return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_coulomb_J_workspace(aux, orb)) return DF3C_E_WORKSPACE;
  return coulomb_J_run(xyz, natom, aux, orb, d, nullptr, J, ws, flags,
                       reinterpret_cast<hipStream_t>(stream));
}

// status word of a call, copied to a caller's device int (one thread)
__global__ void k_copy_status(const int *err, int *status) { *status = *err; }

int df3c_coulomb_J_noalloc(const double *xyz, int32_t natom, const df3c_shells *aux,
                           const df3c_shells *orb, const double *d, double *J, int32_t *status,
                           uint32_t flags, void *stream) {
  if (flags) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !J) return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  if (df3c_coulomb_J_workspace(aux, orb) > DF3C_NOALLOC_SCRATCH_BYTES) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t_no_alloc = true;
  rc = coulomb_J_run(xyz, natom, aux, orb, d, nullptr, J, ds->scratch, DF3C_ASYNC, s);
  t_no_alloc = false;
  if (rc) return rc;
  if (status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<const int *>(ds->scratch), status);
    if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  }
  return DF3C_OK;
}

// ---------------------------------------------------------- Schwarz-type screening
// |(ab|P_m)| <= Q_ab Q_P from positive s-type envelopes of the shells: a
// primitive Cartesian component of l quanta is bounded by M_l(a) e^{-th a r^2}
// (th = 1, M_0 = 1 for l = 0; th = 1/2, M_l = (l/(a e))^{l/2} otherwise),
// and the Coulomb kernel is positive and positive definite, so
//   Q_ab = sum_ij |c_i c_j| M(a_i) M(b_j) e^{-mu_ij AB^2} sqrt((g|g)_ij),
//   Q_P  = t_l sum_k |c_k| M(z_k) sqrt((g|g)_k),
// (g|g) = 2 pi^{5/2} / (g^2 sqrt(2 g)) for the envelope exponents, t_l the
// largest row 1-norm of the solid-harmonic table (1 for a Cartesian shell).
// A pair is kept when Q_ab S_d >= tau with S_d = sum_P Q_P sum_m |d_Pm|: the
// J blocks of the dropped pairs are below tau element by element.
}  // extern "C"
namespace {
__device__ __forceinline__ double env_m(int l, double a) {
  return l == 0 ? 1.0 : pow(double(l) / (a * 2.718281828459045235360287), 0.5 * l);
}
__device__ __forceinline__ double env_theta(int l) { return l == 0 ? 1.0 : 0.5; }
__device__ __forceinline__ double self_rep(double g) {
  return sqrt(34.98683665524972497 / (g * g * sqrt(2.0 * g)));
}
template <int L>
__device__ double solid_row_norm() {
  double t = 0.0;
  for (int m = 0; m < 2 * L + 1; ++m) {
    double r = 0.0;
    for (int q = GenSolid<L>::start[m]; q < GenSolid<L>::start[m + 1]; ++q)
      r += fabs(GenSolid<L>::val[q]);
    t = fmax(t, r);
  }
  return t;
}
__device__ double solid_row_norm_l(int l) {
  switch (l) {
    case 0: return solid_row_norm<0>();
    case 1: return solid_row_norm<1>();
    case 2: return solid_row_norm<2>();
    case 3: return solid_row_norm<3>();
    case 4: return solid_row_norm<4>();
    case 5: return solid_row_norm<5>();
    default: return solid_row_norm<6>();
  }
}

// S_d = sum_P Q_P sum_m |d_Pm| over the aux shells in shell order (one
// workgroup: tiles of PLAN_TPB shells, block scan of the function offsets,
// per-thread partial sums, one fixed-order reduction)
__global__ void __launch_bounds__(PLAN_TPB)
    k_schwarz_fit_sum(const int32_t *l, ShellsDev aux, int32_t n, int32_t pure, const double *d,
                      double *Sd, const int *err) {
  __shared__ int64_t wsum[PLAN_WAVES];
  __shared__ double part[PLAN_TPB];
  if (*err) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int64_t carry = 0;
  double acc = 0.0;
  for (int t0 = 0; t0 < n; t0 += PLAN_TPB) {
    const int s = t0 + tid;
    const int ls = s < n ? min(max(l[s], 0), DF3C_LMAX_AUX) : 0;
    const int nf = s < n ? (pure ? 2 * ls + 1 : (ls + 1) * (ls + 2) / 2) : 0;
    int64_t v = nf;
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t a = __shfl_up(v, o);
      if (lane >= o) v += a;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    int64_t b = carry;
    for (int q = 0; q < w; ++q) b += wsum[q];
    if (s < n) {
      const int64_t o0 = b + v - nf;
      double a1 = 0.0;
      for (int m = 0; m < nf; ++m) a1 += fabs(d[o0 + m]);
      double q = 0.0;
      const int64_t po = aux.prim_off[s];
      for (int k = 0; k < aux.nprim[s]; ++k)
        q += fabs(aux.coefs[po + k]) * env_m(ls, aux.exps[po + k]) *
             self_rep(env_theta(ls) * aux.exps[po + k]);
      acc += (pure ? solid_row_norm_l(ls) : 1.0) * q * a1;
    }
    for (int q = 0; q < PLAN_WAVES; ++q) carry += wsum[q];
    __syncthreads();
  }
  part[tid] = acc;
  __syncthreads();
  for (int o = PLAN_TPB / 2; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  if (tid == 0) *Sd = part[0];
}

__global__ void k_screen_schwarz(const double *xyz, ShellsDev orb, const int32_t *l, int32_t n,
                                 double tau, const double *Sd, uint8_t *mask, const int *err) {
  if (*err) return;
  const double sd = *Sd;
  const int64_t total = int64_t(n) * n;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int sa = int(x / n), sb = int(x - int64_t(sa) * n);
    // the pair's bound from the lower-index shell first: the same arithmetic
    // for (a, b) and (b, a), so the mask is exactly symmetric
    const int s1 = sa >= sb ? sa : sb, s2 = sa >= sb ? sb : sa;
    const int i1 = orb.atom[s1], i2 = orb.atom[s2];
    const double dx = xyz[3 * i1] - xyz[3 * i2], dy = xyz[3 * i1 + 1] - xyz[3 * i2 + 1],
                 dz = xyz[3 * i1 + 2] - xyz[3 * i2 + 2];
    const double ab2 = dx * dx + dy * dy + dz * dz;
    const int l1 = l[s1], l2 = l[s2];
    const double *e1 = orb.exps + orb.prim_off[s1], *c1 = orb.coefs + orb.prim_off[s1];
    const double *e2 = orb.exps + orb.prim_off[s2], *c2 = orb.coefs + orb.prim_off[s2];
    double q = 0.0;
    for (int i = 0; i < orb.nprim[s1]; ++i)
      for (int j = 0; j < orb.nprim[s2]; ++j) {
        const double ea = env_theta(l1) * e1[i], eb = env_theta(l2) * e2[j], g = ea + eb;
        q += fabs(c1[i] * c2[j]) * env_m(l1, e1[i]) * env_m(l2, e2[j]) *
             exp(-ea * eb / g * ab2) * self_rep(g);
      }
    mask[x] = q * sd >= tau ? 1 : 0;
  }
}

}  // namespace
extern "C" {

size_t df3c_screen_pairs_schwarz_workspace(void) { return 512; }

int df3c_screen_pairs_schwarz(const double *xyz, int32_t natom, const df3c_shells *aux,
                              const df3c_shells *orb, const double *d, double tau, uint8_t *mask,
                              void *ws, size_t ws_bytes, uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !mask || !(tau >= 0.0))
    return DF3C_E_ARG;
  if ((aux->pure != 0 && aux->pure != 1) || (orb->pure != 0 && orb->pure != 1))
    return DF3C_E_UNSUPPORTED;
  for (int i = 0; i < aux->nshell; ++i)
    if (aux->l_host[i] < 0 || aux->l_host[i] > DF3C_LMAX_AUX) return DF3C_E_UNSUPPORTED;
  for (int i = 0; i < orb->nshell; ++i)
    if (orb->l_host[i] < 0 || orb->l_host[i] > DF3C_LMAX_ORB) return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_screen_pairs_schwarz_workspace()) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int *err = static_cast<int *>(ws);
  double *Sd = reinterpret_cast<double *>(static_cast<char *>(ws) + 256);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, err, 8, 0);
  check_shells(aux, natom, err, s);
  check_shells(orb, natom, err, s);
  hipLaunchKernelGGL(k_schwarz_fit_sum, dim3(1), dim3(PLAN_TPB), 0, s, aux->l, dev_shells(aux),
                     aux->nshell, aux->pure, d, Sd, err);
  const int64_t total = int64_t(orb->nshell) * orb->nshell;
  if (total > 0)
    hipLaunchKernelGGL(k_screen_schwarz, dim3(int(std::min<int64_t>((total + 255) / 256, 4096))),
                       dim3(256), 0, s, xyz, dev_shells(orb), orb->l, orb->nshell, tau, Sd, mask,
                       err);
  if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  return finish_call(flags, err, s);
}

int df3c_screen_pairs(const double *xyz, int32_t natom, const df3c_shells *orb, double tau,
                      uint8_t *mask, void *stream) {
  if (!xyz || natom <= 0 || !shells_ok(orb) || !mask || !(tau >= 0.0)) return DF3C_E_ARG;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  if (orb->nshell == 0) return DF3C_OK;
  const int64_t total = int64_t(orb->nshell) * orb->nshell;
  const int g = int(std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(k_screen_pairs, dim3(g), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     xyz, dev_shells(orb), orb->nshell, tau, mask);
  return hipGetLastError() == hipSuccess ? DF3C_OK : DF3C_E_HIP;
}

namespace {
size_t masked_core_bytes(const df3c_shells *aux, const df3c_shells *orb) {
  return jplan_bytes(orb->nshell, aux->nshell) + align256(sizeof(unsigned long long) * NLA * NLA) +
         align256(sizeof(int64_t) * size_t(total_class_pairs(orb)));
}
}  // namespace

size_t df3c_coulomb_J_masked_workspace(const df3c_shells *aux, const df3c_shells *orb) {
  if (!shells_ok(aux) || !shells_ok(orb)) return 0;
  return masked_core_bytes(aux, orb) + pure_bytes(orb);
}

int df3c_coulomb_J_masked(const double *xyz, int32_t natom, const df3c_shells *aux,
                          const df3c_shells *orb, const double *d, const uint8_t *mask,
                          double *J, void *ws, size_t ws_bytes, uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !J || !mask)
    return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_coulomb_J_masked_workspace(aux, orb)) return DF3C_E_WORKSPACE;
  return coulomb_J_run(xyz, natom, aux, orb, d, mask, J, ws, flags,
                       reinterpret_cast<hipStream_t>(stream));
}


// ---------------------------------------------------------- two-centre metric
size_t df3c_coulomb_metric_workspace(const df3c_shells *aux) {
  if (!aux) return 0;
  return align256(sizeof(int) * 8) + align256(sizeof(int32_t) * aux->nshell) +
         align256(sizeof(int64_t) * (aux->nshell + 1));
}

int df3c_coulomb_metric(const double *xyz, int32_t natom, const df3c_shells *aux, double *V,
                        void *ws, size_t ws_bytes, uint32_t flags, void *stream) {
  if (flags) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !V) return DF3C_E_ARG;
  if (aux->pure != 0 && aux->pure != 1) return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_coulomb_metric_workspace(aux)) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  // shells grouped by l, function offsets
  std::vector<int32_t> cnt(DF3C_LMAX_AUX + 2, 0), sorted(aux->nshell);
  std::vector<int64_t> off(aux->nshell + 1, 0);
  for (int s = 0; s < aux->nshell; ++s) {
    const int l = aux->l_host[s];
    if (l < 0 || l > DF3C_LMAX_AUX || (!aux->pure && l > 1)) return DF3C_E_UNSUPPORTED;
    cnt[l + 1]++;
    off[s + 1] = off[s] + (aux->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2);
  }
  for (int l = 0; l <= DF3C_LMAX_AUX; ++l) cnt[l + 1] += cnt[l];
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int s = 0; s < aux->nshell; ++s) sorted[fill[aux->l_host[s]]++] = s;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(ws);
  int *err = reinterpret_cast<int *>(w);
  w += align256(sizeof(int) * 8);
  int32_t *sorted_d = reinterpret_cast<int32_t *>(w);
  w += align256(sizeof(int32_t) * aux->nshell);
  int64_t *off_d = reinterpret_cast<int64_t *>(w);
  if (hipMemcpyAsync(sorted_d, sorted.data(), sizeof(int32_t) * aux->nshell,
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(off_d, off.data(), sizeof(int64_t) * (aux->nshell + 1), hipMemcpyHostToDevice,
                     s) != hipSuccess) {
    (void)hipStreamSynchronize(s);  // a copy already queued still reads the host vectors
    return DF3C_E_HIP;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, err, 1, 0);
  check_shells(aux, natom, err, s);
  // the readback also waits for the plan copies, whose host vectors end here
  int word = 0;
  if (read_back(&word, err, sizeof(int), s) != hipSuccess) return DF3C_E_HIP;
  if (word) return DF3C_E_ARG;
  MetArgs a{};
  a.boys = ds->boys;
  a.xyz = xyz;
  a.aux = dev_shells(aux);
  a.aux_off = off_d;
  a.naux = off[aux->nshell];
  a.pure = aux->pure;
  a.V = V;
  for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
    for (int lq = 0; lq <= lp; ++lq) {
      const int np = cnt[lp + 1] - cnt[lp], nq = cnt[lq + 1] - cnt[lq];
      if (!np || !nq) continue;
      a.psh = sorted_d + cnt[lp];
      a.qsh = sorted_d + cnt[lq];
      a.np = np;
      a.nq = nq;
      a.same = (lp == lq);
      a.npair = (lp == lq) ? int64_t(np) * (np + 1) / 2 : int64_t(np) * nq;
      const MetricInfo &mi = g_metric[lp][lq];
      if (mi.fn(a, grid_for(a.npair, mi.ppw, ds->ncu), s) != hipSuccess) return DF3C_E_HIP;
    }
  return DF3C_OK;
}

// ------------------------------------------------------------ adjoint gamma
namespace {
// gamma work items aimed at per class: 4 wavefronts of register items per CU
// Items of the gamma engines for a class of npair shell pairs and np aux
// shells with nacc accumulated components each: nsplit aux subsets (about 8
// aux shells per subset, so that a pair's set-up serves several shells; at
// most 4096 LDS accumulator doubles per item) times nrange ranges of pairs,
// about four wavefronts per SIMD in all.
struct GamRegPlan {
  int32_t nsplit, nps;
  int64_t prange, nrange;
  size_t partial_doubles(int nout) const { return size_t(nrange) * nsplit * nps * nout; }
};
GamRegPlan gam_reg_plan(int64_t npair, int np, int nacc, int ncu, int npsmax) {
  GamRegPlan g;
  const int64_t target = int64_t(ncu) * 16;
  const int lo = int((int64_t(np) * nacc + 4095) / 4096);
  g.nsplit = std::max(lo, std::min(std::max(1, np / 8), 64));
  // at most npsmax aux shells per subset (the LDS accumulators of the register
  // engine with the primitive pairs outermost)
  if (npsmax > 0) g.nsplit = std::max(g.nsplit, (np + npsmax - 1) / npsmax);
  g.nps = (np + g.nsplit - 1) / g.nsplit;
  const int64_t rounds = (npair + 63) / 64;
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(rounds, target / g.nsplit));
  g.prange = (rounds + want - 1) / want * 64;
  g.nrange = (npair + g.prange - 1) / g.prange;
  return g;
}

// register engine: gamma[aux function] += sum over the pair ranges, in order.
// Threads follow the partials' own layout (f = (subset, shell of the subset,
// component) within a range), so every range's reads are contiguous.
__global__ void k_gam_reduce_r(const double *partial, int32_t np, int32_t nsplit, int32_t nps,
                               int64_t nrange, int32_t nout, const int32_t *psh,
                               const int64_t *aux_off, double *gamma, const int *err) {
  if (*err) return;
  const int nf = nsplit * nps * nout;  // doubles of one range's partial
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
    const int t = f / nout, m = f - t * nout;
    const int sub = t / nps, k = t - sub * nps;
    const int ip = k * nsplit + sub;
    if (ip >= np) continue;
    double v = 0.0;
    for (int64_t r = 0; r < nrange; ++r) v += partial[r * nf + f];
    gamma[aux_off[psh[ip]] + m] += v;
  }
}

}  // namespace

namespace {
// bytes of one branch's partial buffer: the partials of the largest class plan
size_t gamma_partial_bytes(const df3c_shells *aux, const df3c_shells *orb, int ncu) {
  size_t part = 1;
  int64_t no[DF3C_LMAX_ORB + 1] = {}, na[DF3C_LMAX_AUX + 1] = {};
  for (int s = 0; s < orb->nshell; ++s)
    if (orb->l_host[s] >= 0 && orb->l_host[s] <= DF3C_LMAX_ORB) ++no[orb->l_host[s]];
  for (int s = 0; s < aux->nshell; ++s)
    if (aux->l_host[s] >= 0 && aux->l_host[s] <= DF3C_LMAX_AUX) ++na[aux->l_host[s]];
  for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
    for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        if (!na[lp] || !no[la] || !no[lb]) continue;
        const int64_t npair = la == lb ? no[la] * (no[la] + 1) / 2 : no[la] * no[lb];
        const int nout = aux->pure ? 2 * lp + 1 : (lp + 1) * (lp + 2) / 2;
        const int nacc = (lp + 1) * (lp + 2) / 2;
        const GamRegPlan gp = gam_reg_plan(npair, int(na[lp]), nacc, ncu, gam_nps_cap(lp));
        part = std::max(part, gp.partial_doubles(nout));
      }
  return align256(sizeof(double) * part);
}
}  // namespace

size_t df3c_coulomb_gamma_workspace(const df3c_shells *aux, const df3c_shells *orb) {
  if (!shells_ok(aux) || !shells_ok(orb)) return 0;
  DevState *ds = nullptr;
  if (init_device(&ds)) return 0;
  // one partial buffer per concurrent branch
  return jplan_bytes(orb->nshell, aux->nshell) + NBRANCH * gamma_partial_bytes(aux, orb, ds->ncu) +
         pullback_bytes(orb);
}

int df3c_coulomb_gamma(const double *xyz, int32_t natom, const df3c_shells *aux,
                       const df3c_shells *orb, const double *D, double *gamma, void *ws,
                       size_t ws_bytes, uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !D || !gamma) return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  const size_t need = df3c_coulomb_gamma_workspace(aux, orb);
  if (!ws || ws_bytes < need) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  HostPlan p;
  if ((rc = host_plan(aux, orb, p))) return rc;
  if (orb->pure && orb->nshell >= (1 << 27)) return DF3C_E_UNSUPPORTED;  // rows packed shell << 4
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DevPlan dp = carve_plan(ws, orb->nshell, aux->nshell);
  int32_t *aux_sorted = dp.aux_sorted;
  int64_t *aux_off = dp.aux_off;
  double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                               jplan_bytes(orb->nshell, aux->nshell));
  // solid-harmonic orbital shells: the engines contract with D_cart = T_a^T D T_b
  // (the pull-back sits at the end of the workspace)
  PullBack pb;
  if (orb->pure)
    pb = carve_pullback(orb, static_cast<char *>(ws) + need - pullback_bytes(orb), p.nao);
  if (launch_plan(dp, p, aux, orb, natom, nullptr, orb->pure ? pb.cmap : nullptr,
                  orb->pure ? pb.poff : nullptr, s) != hipSuccess)
    return DF3C_E_HIP;
  // aux-shell records (no d') for the register engine's aux loop
  if (launch_aux_records(dp.aux_sorted, aux->nshell, aux, xyz, dp.aux_off, nullptr, dp.arec, s,
                         dp.err) != hipSuccess)
    return DF3C_E_HIP;
  hipLaunchKernelGGL(k_zero_f64, dim3(int(std::min<int64_t>((p.naux + 255) / 256, 4096))),
                     dim3(256), 0, s, gamma, p.naux);
  if (orb->pure) {
    if (pull_back_cart(orb, D, pb, p.nao, p.npure, dp.err, s) != hipSuccess) return DF3C_E_HIP;
    D = pb.Gc;
  }
  GamArgs a{};
  a.boys = ds->boys;
  a.xyz = xyz;
  a.aux = dev_shells(aux);
  a.orb = dev_shells(orb);
  a.ao_off = dp.ao_off;
  a.D = D;
  a.nao = p.nao;
  a.pure = aux->pure;
  a.err = dp.err;
  // The classes of one aux l write disjoint gamma entries from those of any
  // other: the L_P groups run on NBRANCH concurrent streams forked from and
  // joined back to s, each branch with its own partial buffer, and inside a
  // group the (l_a, l_b) classes keep their order (gamma is bitwise the
  // one-stream result).  Groups go to branches longest first by a work model.
  const size_t part_stride = gamma_partial_bytes(aux, orb, ds->ncu);
  if ((rc = ensure_branches(ds))) return rc;
  std::lock_guard<std::mutex> branch_lock(g_branch_mu);
  int branch_of[DF3C_LMAX_AUX + 1] = {};
  {
    double gcost[DF3C_LMAX_AUX + 1] = {}, load[NBRANCH] = {};
    for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
      for (int la = 0; la <= DF3C_LMAX_ORB; ++la)
        for (int lb = 0; lb <= la; ++lb) {
          const double na = p.orb_start[la + 1] - p.orb_start[la];
          const double nb = p.orb_start[lb + 1] - p.orb_start[lb];
          gcost[lp] += (la == lb ? na * (na + 1) / 2 : na * nb) *
                       double(p.aux_start[lp + 1] - p.aux_start[lp]) * (2 * lp + 1) * (la + 1) *
                       (la + 2) * (lb + 1) * (lb + 2);
        }
    int gid[DF3C_LMAX_AUX + 1];
    for (int g = 0; g <= DF3C_LMAX_AUX; ++g) gid[g] = g;
    std::stable_sort(gid, gid + DF3C_LMAX_AUX + 1,
                     [&](int x, int y) { return gcost[x] > gcost[y]; });
    for (int k = 0; k <= DF3C_LMAX_AUX; ++k) {
      int bmin = 0;
      for (int b = 1; b < NBRANCH; ++b)
        if (load[b] < load[bmin]) bmin = b;
      branch_of[gid[k]] = bmin;
      load[bmin] += gcost[gid[k]];
    }
  }
  if (hipEventRecord(ds->fork, s) != hipSuccess) return DF3C_E_HIP;
  for (int b = 0; b < NBRANCH - 1; ++b)
    if (hipStreamWaitEvent(ds->side[b], ds->fork, 0) != hipSuccess) return DF3C_E_HIP;
  int brc = DF3C_OK;
  for (int lp = 0; lp <= DF3C_LMAX_AUX && !brc; ++lp) {
    const int np = p.aux_start[lp + 1] - p.aux_start[lp];
    if (!np) continue;
    const int nout = aux->pure ? 2 * lp + 1 : (lp + 1) * (lp + 2) / 2;
    const int br = branch_of[lp];
    hipStream_t bs = br == 0 ? s : ds->side[br - 1];
    double *bpartial = reinterpret_cast<double *>(reinterpret_cast<char *>(partial) +
                                                  size_t(br) * part_stride);
    a.partial = bpartial;
    a.psh = aux_sorted + p.aux_start[lp];
    a.arec = dp.arec + int64_t(p.aux_start[lp]) * AREC;
    a.np = np;
    for (int la = 0; la <= DF3C_LMAX_ORB && !brc; ++la)
      for (int lb = 0; lb <= la && !brc; ++lb) {
        const int na = p.orb_start[la + 1] - p.orb_start[la];
        const int nb = p.orb_start[lb + 1] - p.orb_start[lb];
        if (!na || !nb) continue;
        a.ash = dp.orb_sorted + p.orb_start[la];
        a.bsh = dp.orb_sorted + p.orb_start[lb];
        a.na = na;
        a.nb = nb;
        a.same = (la == lb);
        a.npair = (la == lb) ? int64_t(na) * (na + 1) / 2 : int64_t(na) * nb;
        const ClassInfo &ci = g_cls[lp][la][lb];
        const int c = (lp * NLA + la) * NLA + lb;
        // items (range of pairs, subset of the aux shells) on the register
        // engine or the gamma engine; partials added per class in order
        const GamRegPlan gp =
            gam_reg_plan(a.npair, np, (lp + 1) * (lp + 2) / 2, ds->ncu, gam_nps_cap(lp));
        a.nsplit = gp.nsplit;
        a.nps = gp.nps;
        a.prange = gp.prange;
        a.nrange = gp.nrange;
        const int grid = int(gp.nrange * gp.nsplit);
        if (timed(DF3C_KERNEL_GAMMA, c, bs, [&] { return ci.gam(a, grid, bs); }) != hipSuccess) {
          brc = DF3C_E_HIP;
          break;
        }
        const int nred = gp.nsplit * gp.nps * nout;
        hipLaunchKernelGGL(k_gam_reduce_r, dim3((nred + 255) / 256), dim3(256), 0, bs, bpartial,
                           np, gp.nsplit, gp.nps, gp.nrange, nout, a.psh, aux_off, gamma, dp.err);
      }
  }
  // join every branch back to s, also after a failed launch
  for (int b = 0; b < NBRANCH - 1; ++b)
    if (hipEventRecord(ds->join[b], ds->side[b]) != hipSuccess ||
        hipStreamWaitEvent(s, ds->join[b], 0) != hipSuccess)
      return DF3C_E_HIP;
  if (brc) return brc;
  return finish_call(flags, dp.err, s);
}

// ----------------------------------------------------------------- J gradient
namespace {
constexpr int GRAD_GRID_PER_CU = 16;    // workgroups per CU of every gradient launch
constexpr int GRAD_MAX_TPB = 1;         // teams per workgroup of the gradient kernels
int grad_slots(int ncu) { return ncu * GRAD_GRID_PER_CU * GRAD_MAX_TPB; }

// Aux-shell subsets per shell pair of a gradient class: a class of few pairs
// (or few pairs per wavefront) is split into pairs x subsets work items until
// about four waves per SIMD are available (at most 16 subsets, each with at
// least the class's min_aux aux shells, since every item redoes the pair's
// set-up).
int grad_split(const GradInfo &gi, int64_t npair, int np, int ncu) {
  const int64_t target = int64_t(ncu) * 16;
  auto waves = [&](int k) { return (npair + gi.ppw - 1) / gi.ppw * k * gi.wpb; };
  int n = 1;
  while (n < 16 && 2 * n * gi.min_aux <= np && waves(n) < target) n *= 2;
  return n;
}
}  // namespace

size_t df3c_coulomb_J_grad_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                     int32_t natom) {
  if (!shells_ok(aux) || !shells_ok(orb) || natom < 0) return 0;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  return jplan_bytes(orb->nshell, aux->nshell) +
         align256(sizeof(double) * size_t(grad_slots(ncu)) * 3 * size_t(natom)) +
         pullback_bytes(orb);
}

namespace {
// The J gradient over all pairs (mask null) or over the pairs a mask keeps;
// asynchronous like coulomb_J_run (device plan, status word, device counts).
int grad_run(const double *xyz, int32_t natom, const df3c_shells *aux, const df3c_shells *orb,
             const double *d, const double *G, const uint8_t *mask, double *grad, void *ws,
             size_t ws_bytes, uint32_t flags, hipStream_t s, int32_t atom_base = 0) {
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  const int nslot = grad_slots(ds->ncu);
  const size_t base_need = jplan_bytes(orb->nshell, aux->nshell) +
                           align256(sizeof(double) * size_t(nslot) * 3 * size_t(natom));
  const size_t core = base_need + (mask ? align256(sizeof(unsigned long long) * NLA * NLA) +
                                              align256(sizeof(int64_t) * size_t(total_class_pairs(orb)))
                                        : 0);
  if (!ws || ws_bytes < core + pullback_bytes(orb)) return DF3C_E_WORKSPACE;
  HostPlan p;
  if ((rc = host_plan(aux, orb, p))) return rc;
  for (int l = DF3C_LMAX_GRAD_ORB + 1; l <= DF3C_LMAX_ORB; ++l)
    if (p.orb_start[l + 1] > p.orb_start[l]) return DF3C_E_UNSUPPORTED;
  if (orb->pure && orb->nshell >= (1 << 27)) return DF3C_E_UNSUPPORTED;  // rows packed shell << 4
  // the per-workgroup atom arrays must fit the LDS of every launched class
  for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
    for (int la = 0; la <= DF3C_LMAX_GRAD_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        if (!p.ca.n[lp] || !p.co.n[la] || !p.co.n[lb]) continue;
        const GradInfo &gi = g_grad[lp][la][lb];
        if (gi.tpb * (gi.team + 3 * int64_t(natom)) * 8 > 160 * 1024) return DF3C_E_UNSUPPORTED;
      }
  const DevPlan dp = carve_plan(ws, orb->nshell, aux->nshell);
  double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                               jplan_bytes(orb->nshell, aux->nshell));
  // masked only: kept-pair counters and lists of the (l_a, l_b) classes
  unsigned long long *pcount = nullptr;
  int64_t *plist = nullptr;
  if (mask) {
    char *m = static_cast<char *>(ws) + base_need;
    pcount = reinterpret_cast<unsigned long long *>(m);
    plist = reinterpret_cast<int64_t *>(m + align256(sizeof(unsigned long long) * NLA * NLA));
  }
  // solid-harmonic orbital shells: the engines take G_cart = T_a^T G T_b
  PullBack pb;
  if (orb->pure) pb = carve_pullback(orb, static_cast<char *>(ws) + core, p.nao);
  if (launch_plan(dp, p, aux, orb, natom, nullptr, orb->pure ? pb.cmap : nullptr,
                  orb->pure ? pb.poff : nullptr, s, atom_base) != hipSuccess)
    return DF3C_E_HIP;
  const int64_t npart = int64_t(nslot) * 3 * natom;
  hipLaunchKernelGGL(k_zero_f64, dim3(int(std::min<int64_t>((npart + 255) / 256, 4096))),
                     dim3(256), 0, s, partial, npart);
  if (orb->pure) {
    if (pull_back_cart(orb, G, pb, p.nao, p.npure, dp.err, s) != hipSuccess) return DF3C_E_HIP;
    G = pb.Gc;
  }
  GradArgs a{};
  a.boys = ds->boys;
  a.xyz = xyz;
  a.aux = dev_shells(aux);
  a.orb = dev_shells(orb);
  a.ao_off = dp.ao_off;
  a.aux_off = dp.aux_off;
  a.d = d;
  a.G = G;
  a.nao = p.nao;
  a.pure = aux->pure;
  a.natom = natom;
  a.partial = partial;
  a.err = dp.err;
  a.atom_base = atom_base;
  // masked: compact the kept pairs of every class on the device; launches
  // are sized for the whole class and the kernels read the kept count
  int64_t loff[NLA][NLA] = {};
  if (mask) {
    int64_t o = 0;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int *>(pcount),
                       2 * NLA * NLA, 0);
    CompactJobs jobs{};
    int nj = 0;
    for (int la = 0; la <= DF3C_LMAX_GRAD_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        loff[la][lb] = o;
        const int na = p.orb_start[la + 1] - p.orb_start[la];
        const int nb = p.orb_start[lb + 1] - p.orb_start[lb];
        if (!na || !nb) continue;
        const int64_t npair = (la == lb) ? int64_t(na) * (na + 1) / 2 : int64_t(na) * nb;
        jobs.j[nj++] = CompactJob{dp.orb_sorted + p.orb_start[la], dp.orb_sorted + p.orb_start[lb],
                                  nb, int(la == lb), npair, plist + o, pcount + la * NLA + lb};
        o += npair;
      }
    if (nj) {
      hipLaunchKernelGGL(k_pair_compact, dim3(nj), dim3(COMPACT_TPB), 0, s, jobs, mask,
                         orb->nshell, dp.err);
      if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
    }
  }
  // without DF3C_ASYNC the kept counts are read back once and size the launches
  unsigned long long kept[NLA * NLA] = {};
  const bool sized = mask && !(flags & DF3C_ASYNC);
  if (sized && read_back(kept, pcount, sizeof(kept), s) != hipSuccess) return DF3C_E_HIP;
  // The (l_a, l_b) groups run on NBRANCH concurrent streams forked from and
  // joined back to s; each branch owns a quarter of the partial slots (the
  // workgroups of its launches add into those), and inside a branch the
  // classes keep their order, so every slot sums the same contributions in
  // the same sequence on every call and the final fixed-order reduction is
  // reproducible bit for bit.
  auto prep = [&](int la, int lb) {
    const int na = p.orb_start[la + 1] - p.orb_start[la];
    const int nb = p.orb_start[lb + 1] - p.orb_start[lb];
    if (!na || !nb) return false;
    a.ash = dp.orb_sorted + p.orb_start[la];
    a.bsh = dp.orb_sorted + p.orb_start[lb];
    a.na = na;
    a.nb = nb;
    a.same = (la == lb);
    a.npair = (la == lb) ? int64_t(na) * (na + 1) / 2 : int64_t(na) * nb;
    if (mask) {
      a.plist = plist + loff[la][lb];
      a.pcount = reinterpret_cast<const int64_t *>(pcount + la * NLA + lb);
      if (sized) a.npair = int64_t(kept[la * NLA + lb]);  // the kernels read *pcount
    }
    return a.npair > 0;
  };
  if ((rc = ensure_branches(ds))) return rc;
  std::lock_guard<std::mutex> branch_lock(g_branch_mu);
  int branch_of[NLA * NLA] = {};
  {
    double gcost[NLA * NLA] = {}, load[NBRANCH] = {};
    for (int la = 0; la <= DF3C_LMAX_GRAD_ORB; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        if (!prep(la, lb)) continue;
        for (int lp = 0; lp <= DF3C_LMAX_AUX; ++lp)
          gcost[la * NLA + lb] += double(a.npair) * double(p.aux_start[lp + 1] - p.aux_start[lp]) *
                                  (lp + 1) * (lp + 2) * (la + 1) * (la + 2) * (lb + 1) * (lb + 2);
      }
    int gid[NLA * NLA];
    for (int g = 0; g < NLA * NLA; ++g) gid[g] = g;
    std::stable_sort(gid, gid + NLA * NLA, [&](int x, int y) { return gcost[x] > gcost[y]; });
    for (int k = 0; k < NLA * NLA; ++k) {
      int bmin = 0;
      for (int b = 1; b < NBRANCH; ++b)
        if (load[b] < load[bmin]) bmin = b;
      branch_of[gid[k]] = bmin;
      load[bmin] += gcost[gid[k]];
    }
  }
  const int slots_b = nslot / NBRANCH;
  if (hipEventRecord(ds->fork, s) != hipSuccess) return DF3C_E_HIP;
  for (int b = 0; b < NBRANCH - 1; ++b)
    if (hipStreamWaitEvent(ds->side[b], ds->fork, 0) != hipSuccess) return DF3C_E_HIP;
  int brc = DF3C_OK;
  for (int lp = 0; lp <= DF3C_LMAX_AUX && !brc; ++lp) {
    const int np = p.aux_start[lp + 1] - p.aux_start[lp];
    if (!np) continue;
    a.psh = dp.aux_sorted + p.aux_start[lp];
    a.np = np;
    for (int la = 0; la <= DF3C_LMAX_GRAD_ORB && !brc; ++la)
      for (int lb = 0; lb <= la && !brc; ++lb) {
        if (!prep(la, lb)) continue;
        const int br = branch_of[la * NLA + lb];
        hipStream_t bs = br == 0 ? s : ds->side[br - 1];
        a.partial = partial + int64_t(br) * slots_b * 3 * natom;
        const GradInfo &gi = g_grad[lp][la][lb];
        const int lds = gi.tpb * (gi.team + 3 * natom) * 8;
        a.nsplit = grad_split(gi, a.npair, np, ds->ncu);
        const int64_t blocks = (a.npair + gi.ppw - 1) / gi.ppw * a.nsplit;
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(blocks, slots_b)));
        if (timed(DF3C_KERNEL_GRAD, (lp * NLA + la) * NLA + lb, bs,
                  [&] { return gi.gfn(a, grid, lds, bs); }) != hipSuccess)
          brc = DF3C_E_HIP;
      }
  }
  // join every branch back to s, also after a failed launch
  for (int b = 0; b < NBRANCH - 1; ++b)
    if (hipEventRecord(ds->join[b], ds->side[b]) != hipSuccess ||
        hipStreamWaitEvent(s, ds->join[b], 0) != hipSuccess)
      return DF3C_E_HIP;
  if (brc) return brc;
  const int n = 3 * natom;
  hipLaunchKernelGGL(k_reduce_partial, dim3((n + 255) / 256), dim3(256), 0, s, partial, nslot, n,
                     grad);
  if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  return finish_call(flags, dp.err, s);
}
}  // namespace

int df3c_coulomb_J_grad(const double *xyz, int32_t natom, const df3c_shells *aux,
                        const df3c_shells *orb, const double *d, const double *G, double *grad,
                        void *ws, size_t ws_bytes, uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !G || !grad)
    return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  return grad_run(xyz, natom, aux, orb, d, G, nullptr, grad, ws, ws_bytes, flags,
                  reinterpret_cast<hipStream_t>(stream));
}

size_t df3c_coulomb_J_grad_masked_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                            int32_t natom) {
  if (!shells_ok(aux) || !shells_ok(orb) || natom < 0) return 0;
  return df3c_coulomb_J_grad_workspace(aux, orb, natom) +
         align256(sizeof(unsigned long long) * NLA * NLA) +
         align256(sizeof(int64_t) * size_t(total_class_pairs(orb)));
}

int df3c_coulomb_J_grad_masked(const double *xyz, int32_t natom, const df3c_shells *aux,
                               const df3c_shells *orb, const double *d, const double *G,
                               const uint8_t *mask, double *grad, void *ws, size_t ws_bytes,
                               uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !G || !grad || !mask)
    return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  return grad_run(xyz, natom, aux, orb, d, G, mask, grad, ws, ws_bytes, flags,
                  reinterpret_cast<hipStream_t>(stream));
}


// ------------------------------------------------------- batched J gradient
namespace {
__global__ void k_or_status(const int *err, int *acc) {
  if (threadIdx.x == 0 && *err) atomicOr(acc, *err);
}

// sub-basis of the shells [s0, s1) (prim_off and atom stay global)
df3c_shells shell_range(const df3c_shells *b, int s0, int s1) {
  df3c_shells r = *b;
  r.nshell = s1 - s0;
  r.l_host = b->l_host + s0;
  r.l = b->l + s0;
  r.nprim = b->nprim + s0;
  r.prim_off = b->prim_off + s0;
  r.atom = b->atom + s0;
  r.nprim_host = b->nprim_host ? b->nprim_host + s0 : nullptr;
  return r;
}

bool batch_ranges_ok(int nmol, const int32_t *r, int32_t total) {
  if (!r || r[0] != 0 || r[nmol] != total) return false;
  for (int m = 0; m < nmol; ++m)
    if (r[m + 1] < r[m]) return false;
  return true;
}
}  // namespace

size_t df3c_coulomb_J_grad_batched_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                             int32_t nmol, const int32_t *mol_orb,
                                             const int32_t *mol_aux, const int32_t *mol_atom) {
  if (!shells_ok(aux) || !shells_ok(orb) || nmol <= 0 || !mol_orb || !mol_aux || !mol_atom)
    return 0;
  size_t w = 0;
  for (int m = 0; m < nmol; ++m) {
    const df3c_shells am = shell_range(aux, mol_aux[m], mol_aux[m + 1]);
    const df3c_shells om = shell_range(orb, mol_orb[m], mol_orb[m + 1]);
    w = std::max(w, df3c_coulomb_J_grad_workspace(&am, &om, mol_atom[m + 1] - mol_atom[m]));
  }
  return 256 + w;
}

int df3c_coulomb_J_grad_batched(const double *xyz, int32_t natom, const df3c_shells *aux,
                                const df3c_shells *orb, int32_t nmol, const int32_t *mol_orb,
                                const int32_t *mol_aux, const int32_t *mol_atom, const double *d,
                                const double *G, double *grad, void *ws, size_t ws_bytes,
                                uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !G || !grad || nmol <= 0)
    return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  if (!batch_ranges_ok(nmol, mol_orb, orb->nshell) || !batch_ranges_ok(nmol, mol_aux, aux->nshell) ||
      !batch_ranges_ok(nmol, mol_atom, natom))
    return DF3C_E_ARG;
  for (int s = 0; s < orb->nshell; ++s)
    if (orb->l_host[s] < 0 || orb->l_host[s] > DF3C_LMAX_ORB) return DF3C_E_UNSUPPORTED;
  for (int s = 0; s < aux->nshell; ++s)
    if (aux->l_host[s] < 0 || aux->l_host[s] > DF3C_LMAX_AUX) return DF3C_E_UNSUPPORTED;
  const size_t need = df3c_coulomb_J_grad_batched_workspace(aux, orb, nmol, mol_orb, mol_aux,
                                                            mol_atom);
  if (!ws || ws_bytes < need) return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int *status = static_cast<int *>(ws);
  char *mws = static_cast<char *>(ws) + 256;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, status, 8, 0);
  // per molecule: its shells, fitting coefficients, G block (molecule m's
  // nao_m x nao_m matrix at offset sum_{m' < m} nao_m'^2) and atoms; the
  // gradient engines run on the molecule's own atom range
  int64_t doff = 0, goff = 0;
  for (int m = 0; m < nmol; ++m) {
    const df3c_shells am = shell_range(aux, mol_aux[m], mol_aux[m + 1]);
    const df3c_shells om = shell_range(orb, mol_orb[m], mol_orb[m + 1]);
    int64_t naux_m = 0, nao_m = 0;
    for (int q = 0; q < am.nshell; ++q) {
      const int l = am.l_host[q];
      naux_m += aux->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2;
    }
    for (int q = 0; q < om.nshell; ++q) {
      const int l = om.l_host[q];
      nao_m += orb->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2;
    }
    const int a0 = mol_atom[m], na = mol_atom[m + 1] - mol_atom[m];
    if (na > 0) {
      rc = grad_run(xyz + 3 * int64_t(a0), na, &am, &om, d + doff, G + goff, nullptr,
                    grad + 3 * int64_t(a0), mws, ws_bytes - 256, DF3C_ASYNC, s, a0);
      if (rc) {
        (void)hipStreamSynchronize(s);
        return rc;
      }
      hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, s, reinterpret_cast<const int *>(mws),
                         status);
    }
    doff += naux_m;
    goff += nao_m * nao_m;
  }
  if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  return finish_call(flags, status, s);
}

// --------------------------------------------------------------- batched DF-J
namespace {
// solid-harmonic orbital shells: per molecule, where its pure rows, its
// Cartesian J (in the workspace) and its pure J (the caller's) lie
struct PMol {
  int64_t pbase, np, jpbase, jcbase, nc, ao_base;
};

struct BPlan {
  std::vector<int32_t> orb_sorted, aux_sorted;  // per molecule, grouped by l
  std::vector<int64_t> ao_off, aux_off;
  std::vector<JSeg> seg;                         // all classes, class-major
  int32_t cls_seg0[NCLS + 1] = {};               // segment range of every class
  int64_t cls_items[NCLS] = {};
  std::vector<int64_t> jbase, nao_m, ao_base;
  int64_t jtotal = 0;                            // Cartesian J doubles of all molecules
  // orb->pure = 1: pure rows (shell << 4 | m) of all molecules, per-molecule records
  std::vector<int32_t> prow;
  std::vector<PMol> pmol;
  int64_t np_max = 0;
};

size_t bplan_bytes(int64_t norb, int64_t naux, int64_t nmol) {
  return align256(sizeof(int) * 8) + align256(sizeof(int32_t) * norb) +
         align256(sizeof(int32_t) * naux) + align256(sizeof(int64_t) * (norb + 1)) +
         align256(sizeof(int64_t) * (naux + 1)) + align256(sizeof(JSeg) * nmol * NCLS) +
         align256(sizeof(unsigned long long) * NCLS) + align256(sizeof(double) * AREC * naux);
}

// extra workspace of solid-harmonic orbital shells: the Cartesian J of every
// molecule, the pure row map and the per-molecule records
size_t bplan_pure_bytes(const df3c_shells *orb, int32_t nmol, const int32_t *mol_orb) {
  int64_t jc = 0, np = 0;
  for (int m = 0; m < nmol; ++m) {
    int64_t nc = 0;
    for (int s = mol_orb[m]; s < mol_orb[m + 1]; ++s) {
      const int l = orb->l_host[s];
      nc += (l + 1) * (l + 2) / 2;
      np += 2 * l + 1;
    }
    jc += nc * nc;
  }
  return align256(sizeof(double) * jc) + align256(sizeof(int32_t) * np) +
         align256(sizeof(PMol) * nmol);
}

// J[m] pure = T_a Jc[m] T_b^T over the pure rows of molecule m (blockIdx.y
// strides over molecules; an element above the diagonal is evaluated as its
// mirror, as in k_bra_pure)
__global__ void k_bra_pure_mol(const double *Jc, const PMol *pm, int32_t nmol,
                               const int32_t *prow, const int64_t *ao_off, const int32_t *lsh,
                               double *J, const int *err) {
  if (*err) return;
  for (int m = blockIdx.y; m < nmol; m += gridDim.y) {
    const PMol q = pm[m];
    const int64_t total = q.np * q.np;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
      int64_t r = x / q.np, c = x - r * q.np;
      if (r < c) {
        const int64_t t = r;
        r = c;
        c = t;
      }
      const int sa = prow[q.pbase + r] >> 4, ma = prow[q.pbase + r] & 15;
      const int sb = prow[q.pbase + c] >> 4, mb = prow[q.pbase + c] & 15;
      int na, nb;
      const int16_t *ca, *cb;
      const double *va, *vb;
      solid_row_l(lsh[sa], ma, na, ca, va);
      solid_row_l(lsh[sb], mb, nb, cb, vb);
      const double *row = Jc + q.jcbase + (ao_off[sa] - q.ao_base) * q.nc + (ao_off[sb] - q.ao_base);
      double v = 0.0;
      for (int i = 0; i < na; ++i) {
        double t = 0.0;
        for (int j = 0; j < nb; ++j) t += vb[j] * row[int64_t(ca[i]) * q.nc + cb[j]];
        v += va[i] * t;
      }
      J[q.jpbase + x] = v;
    }
  }
}

// Orbital shells of one l in order of decreasing contraction degree (stable),
// the order of the device plans: the kernels give one lane or one team to a
// shell pair and loop over its primitive pairs, so pairs that share a
// wavefront should have equal Ka Kb.
void sort_by_contraction(const df3c_shells *orb, int32_t *first, int32_t *last) {
  if (!orb->nprim_host) return;
  std::stable_sort(first, last, [orb](int32_t x, int32_t y) {
    return orb->nprim_host[x] > orb->nprim_host[y];
  });
}

int make_bplan(const df3c_shells *aux, const df3c_shells *orb, int nmol, const int32_t *mo,
               const int32_t *ma, BPlan &p) {
  if (!aux->l_host || !orb->l_host || !mo || !ma || nmol <= 0) return DF3C_E_ARG;
  if (mo[0] != 0 || ma[0] != 0 || mo[nmol] != orb->nshell || ma[nmol] != aux->nshell)
    return DF3C_E_ARG;
  for (int m = 0; m < nmol; ++m)
    if (mo[m + 1] < mo[m] || ma[m + 1] < ma[m]) return DF3C_E_ARG;
  p.ao_off.assign(orb->nshell + 1, 0);
  p.aux_off.assign(aux->nshell + 1, 0);
  for (int s = 0; s < orb->nshell; ++s) {
    const int l = orb->l_host[s];
    if (l < 0 || l > DF3C_LMAX_ORB) return DF3C_E_UNSUPPORTED;
    p.ao_off[s + 1] = p.ao_off[s] + (l + 1) * (l + 2) / 2;
  }
  for (int s = 0; s < aux->nshell; ++s) {
    const int l = aux->l_host[s];
    if (l < 0 || l > DF3C_LMAX_AUX || (!aux->pure && l > 1)) return DF3C_E_UNSUPPORTED;
    p.aux_off[s + 1] = p.aux_off[s] + (aux->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2);
  }
  // per molecule: shells grouped by l
  std::vector<std::array<int32_t, DF3C_LMAX_ORB + 2>> ost(nmol);
  std::vector<std::array<int32_t, DF3C_LMAX_AUX + 2>> ast(nmol);
  p.orb_sorted.clear();
  p.aux_sorted.clear();
  p.jbase.resize(nmol);
  p.nao_m.resize(nmol);
  p.ao_base.resize(nmol);
  int64_t jb = 0;
  for (int m = 0; m < nmol; ++m) {
    for (int l = 0; l <= DF3C_LMAX_ORB; ++l) {
      ost[m][l] = int32_t(p.orb_sorted.size());
      for (int s = mo[m]; s < mo[m + 1]; ++s)
        if (orb->l_host[s] == l) p.orb_sorted.push_back(s);
      sort_by_contraction(orb, p.orb_sorted.data() + ost[m][l], p.orb_sorted.data() + p.orb_sorted.size());
    }
    ost[m][DF3C_LMAX_ORB + 1] = int32_t(p.orb_sorted.size());
    for (int l = 0; l <= DF3C_LMAX_AUX; ++l) {
      ast[m][l] = int32_t(p.aux_sorted.size());
      for (int s = ma[m]; s < ma[m + 1]; ++s)
        if (aux->l_host[s] == l) p.aux_sorted.push_back(s);
    }
    ast[m][DF3C_LMAX_AUX + 1] = int32_t(p.aux_sorted.size());
    p.ao_base[m] = p.ao_off[mo[m]];
    p.nao_m[m] = p.ao_off[mo[m + 1]] - p.ao_off[mo[m]];
    p.jbase[m] = jb;
    jb += p.nao_m[m] * p.nao_m[m];
  }
  p.jtotal = jb;
  p.prow.clear();
  p.pmol.clear();
  p.np_max = 0;
  if (orb->pure) {
    if (orb->nshell >= (1 << 27)) return DF3C_E_UNSUPPORTED;  // rows packed shell << 4
    int64_t jp = 0;
    for (int m = 0; m < nmol; ++m) {
      PMol q{};
      q.pbase = int64_t(p.prow.size());
      for (int s = mo[m]; s < mo[m + 1]; ++s)
        for (int k = 0; k < 2 * orb->l_host[s] + 1; ++k) p.prow.push_back((s << 4) | k);
      q.np = int64_t(p.prow.size()) - q.pbase;
      q.jpbase = jp;
      q.jcbase = p.jbase[m];
      q.nc = p.nao_m[m];
      q.ao_base = p.ao_base[m];
      jp += q.np * q.np;
      p.np_max = std::max(p.np_max, q.np);
      p.pmol.push_back(q);
    }
  }
  p.seg.clear();
  for (int c = 0; c < NCLS; ++c) {
    p.cls_seg0[c] = int32_t(p.seg.size());
    const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
    int64_t items = 0;
    if (lb <= la)
      for (int m = 0; m < nmol; ++m) {
        const int na = ost[m][la + 1] - ost[m][la], nb = ost[m][lb + 1] - ost[m][lb];
        const int np = ast[m][lp + 1] - ast[m][lp];
        if (!na || !nb || !np) continue;
        JSeg g{};
        g.item0 = items;
        g.npair = (la == lb) ? int64_t(na) * (na + 1) / 2 : int64_t(na) * nb;
        g.jbase = p.jbase[m];
        g.nao = p.nao_m[m];
        g.ao_base = p.ao_base[m];
        g.ash = ost[m][la];
        g.bsh = ost[m][lb];
        g.psh = ast[m][lp];
        g.na = na;
        g.nb = nb;
        g.np = np;
        g.same = (la == lb);
        g.pad = m;  // molecule index
        items += g.npair;
        p.seg.push_back(g);
      }
    p.cls_items[c] = items;
  }
  p.cls_seg0[NCLS] = int32_t(p.seg.size());
  return DF3C_OK;
}

uint64_t fnv(uint64_t h, const void *data, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// A cached executable graph owns the host plan its launches were captured
// from: every call uploads that plan into the caller's workspace before the
// replay (the copies read the entry's memory, which outlives them), so a
// replay never depends on what the workspace held before.  At most
// GRAPH_CACHE entries are kept; the oldest is destroyed first.
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  std::shared_ptr<BPlan> plan;
  uint64_t stamp = 0;
};
constexpr size_t GRAPH_CACHE = 8;
std::unordered_map<uint64_t, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
std::mutex g_graph_mu;

df3c_class_tune default_tune(int c) {
  df3c_class_tune t{};
  t.chunk = 1;
  t.grid_per_cu = 4;
  t.enabled = 1;
  t.order = -int(c / (NLA * NLA));  // high l_P first (the longest classes start early)
  return t;
}
}  // namespace

size_t df3c_coulomb_J_batched_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                        int32_t nmol, const int32_t *mol_orb) {
  if (!aux || !orb || nmol <= 0) return 0;
  if (orb->pure) {
    if (!mol_orb || !orb->l_host || !batch_ranges_ok(nmol, mol_orb, orb->nshell)) return 0;
    return bplan_bytes(orb->nshell, aux->nshell, nmol) + bplan_pure_bytes(orb, nmol, mol_orb);
  }
  return bplan_bytes(orb->nshell, aux->nshell, nmol);
}

int df3c_coulomb_J_batched(const double *xyz, int32_t natom, const df3c_shells *aux,
                           const df3c_shells *orb, int32_t nmol, const int32_t *mol_orb,
                           const int32_t *mol_aux, const double *d, double *J,
                           const df3c_class_tune *tune, void *ws, size_t ws_bytes,
                           uint32_t flags, void *stream) {
  if (!xyz || natom <= 0 || !shells_ok(aux) || !shells_ok(orb) || !d || !J || nmol <= 0)
    return DF3C_E_ARG;
  if ((orb->pure != 0 && orb->pure != 1) || (aux->pure != 0 && aux->pure != 1))
    return DF3C_E_UNSUPPORTED;
  if (flags & ~(DF3C_SCHED_PERSISTENT | DF3C_GRAPH | DF3C_ASYNC)) return DF3C_E_ARG;
  if (!mol_orb || !mol_aux || !batch_ranges_ok(nmol, mol_orb, orb->nshell) ||
      !batch_ranges_ok(nmol, mol_aux, aux->nshell))
    return DF3C_E_ARG;
  if (!ws || ws_bytes < df3c_coulomb_J_batched_workspace(aux, orb, nmol, mol_orb))
    return DF3C_E_WORKSPACE;
  DevState *ds = nullptr;
  int rc = init_device(&ds);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  df3c_class_tune tt[NCLS];
  for (int c = 0; c < NCLS; ++c) {
    tt[c] = tune ? tune[c] : default_tune(c);
    if (tt[c].chunk < 1 || tt[c].grid_per_cu < 1) return DF3C_E_ARG;
  }

  // graph cache key: every argument that the captured launches depend on
  uint64_t key = 1469598103934665603ull;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DF3C_E_HIP;
  const void *ptrs[] = {xyz, aux->l, aux->nprim, aux->prim_off, aux->atom, aux->exps, aux->coefs,
                        orb->l, orb->nprim, orb->prim_off, orb->atom, orb->exps, orb->coefs,
                        d, J, ws};
  key = fnv(key, ptrs, sizeof(ptrs));
  const int64_t scal[] = {natom, aux->nshell, orb->nshell, aux->pure, orb->pure, nmol,
                          int64_t(ws_bytes), int64_t(flags), dev};
  key = fnv(key, scal, sizeof(scal));
  key = fnv(key, aux->l_host, sizeof(int32_t) * aux->nshell);
  key = fnv(key, orb->l_host, sizeof(int32_t) * orb->nshell);
  key = fnv(key, mol_orb, sizeof(int32_t) * (nmol + 1));
  key = fnv(key, mol_aux, sizeof(int32_t) * (nmol + 1));
  key = fnv(key, tt, sizeof(tt));
  std::shared_ptr<BPlan> pp;
  hipGraphExec_t hit = nullptr;
  if (flags & DF3C_GRAPH) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
      hit = it->second.exec;
      pp = it->second.plan;
      it->second.stamp = ++g_graph_clock;
    }
  }
  if (!pp) {
    pp = std::make_shared<BPlan>();
    rc = make_bplan(aux, orb, nmol, mol_orb, mol_aux, *pp);
    if (rc) return rc;
  }
  const BPlan &p = *pp;
  char *w = static_cast<char *>(ws);
  int *err = reinterpret_cast<int *>(w);
  w += align256(sizeof(int) * 8);
  int32_t *orb_sorted = reinterpret_cast<int32_t *>(w);
  w += align256(sizeof(int32_t) * orb->nshell);
  int32_t *aux_sorted = reinterpret_cast<int32_t *>(w);
  w += align256(sizeof(int32_t) * aux->nshell);
  int64_t *ao_off = reinterpret_cast<int64_t *>(w);
  w += align256(sizeof(int64_t) * (orb->nshell + 1));
  int64_t *aux_off = reinterpret_cast<int64_t *>(w);
  w += align256(sizeof(int64_t) * (aux->nshell + 1));
  JSeg *segd = reinterpret_cast<JSeg *>(w);
  w += align256(sizeof(JSeg) * nmol * NCLS);
  unsigned long long *ctr = reinterpret_cast<unsigned long long *>(w);
  w += align256(sizeof(unsigned long long) * NCLS);
  double *arec = reinterpret_cast<double *>(w);
  w += align256(sizeof(double) * AREC * aux->nshell);
  // solid-harmonic orbital shells: the engines write the Cartesian J here and
  // one transform per molecule writes the caller's J
  double *Jc = J;
  int32_t *prow = nullptr;
  PMol *pmol = nullptr;
  if (orb->pure) {
    Jc = reinterpret_cast<double *>(w);
    w += align256(sizeof(double) * p.jtotal);
    prow = reinterpret_cast<int32_t *>(w);
    w += align256(sizeof(int32_t) * p.prow.size());
    pmol = reinterpret_cast<PMol *>(w);
    if ((!p.prow.empty() && hipMemcpyAsync(prow, p.prow.data(), sizeof(int32_t) * p.prow.size(),
                                           hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(pmol, p.pmol.data(), sizeof(PMol) * p.pmol.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess) {
      (void)hipStreamSynchronize(s);
      return DF3C_E_HIP;
    }
  }
  if ((!p.orb_sorted.empty() &&
       hipMemcpyAsync(orb_sorted, p.orb_sorted.data(), sizeof(int32_t) * p.orb_sorted.size(),
                      hipMemcpyHostToDevice, s) != hipSuccess) ||
      (!p.aux_sorted.empty() &&
       hipMemcpyAsync(aux_sorted, p.aux_sorted.data(), sizeof(int32_t) * p.aux_sorted.size(),
                      hipMemcpyHostToDevice, s) != hipSuccess) ||
      hipMemcpyAsync(ao_off, p.ao_off.data(), sizeof(int64_t) * p.ao_off.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(aux_off, p.aux_off.data(), sizeof(int64_t) * p.aux_off.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      (!p.seg.empty() && hipMemcpyAsync(segd, p.seg.data(), sizeof(JSeg) * p.seg.size(),
                                        hipMemcpyHostToDevice, s) != hipSuccess)) {
    (void)hipStreamSynchronize(s);  // copies already queued still read the plan
    return DF3C_E_HIP;
  }
  // an error after the plan upload waits for its copies before the plan goes
  auto fail = [&](int r) {
    (void)hipStreamSynchronize(s);
    return r;
  };
  // the descriptors are checked on every call (the kernels read the status
  // word and do nothing when it is set)
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, err, 8, 0);
  check_shells(aux, natom, err, s);
  check_shells(orb, natom, err, s);
  if (hit) {
    if (hipGraphLaunch(hit, s) != hipSuccess) return DF3C_E_HIP;
    return finish_call(flags, err, s);
  }

  if ((flags & DF3C_SCHED_PERSISTENT) && ensure_branches(ds)) return fail(DF3C_E_HIP);
  // the fork / join events are per device (see g_branch_mu)
  std::unique_lock<std::mutex> branch_lock(g_branch_mu, std::defer_lock);
  if (flags & DF3C_SCHED_PERSISTENT) branch_lock.lock();
  // class launch order
  std::vector<int> order;
  for (int c = 0; c < NCLS; ++c)
    if (p.cls_items[c] > 0 && tt[c].enabled) order.push_back(c);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return tt[x].order < tt[y].order; });

  JArgs base{};
  base.boys = ds->boys;
  base.xyz = xyz;
  base.aux = dev_shells(aux);
  base.orb = dev_shells(orb);
  base.ao_off = ao_off;
  base.aux_off = aux_off;
  base.d = d;
  base.pure = aux->pure;
  base.err = err;
  // lanes per pair of the register engine: one value per class from the
  // batch's totals, so that both schedules sum in the same order
  auto class_nsub = [&](int c) {
    const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
    int np_max = 0;
    for (int g = p.cls_seg0[c]; g < p.cls_seg0[c + 1]; ++g) np_max = std::max(np_max, p.seg[g].np);
    return reg_split(g_cls[lp][la][lb], p.cls_items[c], np_max, ds->ncu);
  };

  base.arec = arec;

  auto enqueue = [&]() -> int {
    hipLaunchKernelGGL(k_zero_f64, dim3(int(std::min<int64_t>((p.jtotal + 255) / 256, 4096))),
                       dim3(256), 0, s, Jc, p.jtotal);
    if (launch_aux_records(aux_sorted, int64_t(p.aux_sorted.size()), aux, xyz, aux_off, d, arec,
                           s, err) != hipSuccess)
      return DF3C_E_HIP;
    if (flags & DF3C_SCHED_PERSISTENT) {
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, reinterpret_cast<int *>(ctr),
                         2 * NCLS, 0);
      // Classes of different (l_a, l_b) write disjoint J blocks, so the
      // (l_a, l_b) groups run on NBRANCH concurrent streams (forked from and
      // joined back to s, also under capture: the graph gets parallel
      // branches); inside a group the L_P classes keep the order of `order`,
      // so every J element sums its classes in the same sequence as the
      // per-class schedule (bitwise equal).  Groups go to branches longest
      // first by a work model (items x functions of the class).
      int branch_of[NLA * NLA];
      {
        double gcost[NLA * NLA] = {}, load[NBRANCH] = {};
        for (int c : order) {
          const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
          gcost[la * NLA + lb] += double(p.cls_items[c]) * (2 * lp + 1) * (la + 1) * (la + 2) *
                                  (lb + 1) * (lb + 2);
        }
        int gid[NLA * NLA];
        for (int g = 0; g < NLA * NLA; ++g) gid[g] = g;
        std::stable_sort(gid, gid + NLA * NLA, [&](int x, int y) { return gcost[x] > gcost[y]; });
        for (int k = 0; k < NLA * NLA; ++k) {
          const int g = gid[k];
          int bmin = 0;
          for (int b = 1; b < NBRANCH; ++b)
            if (load[b] < load[bmin]) bmin = b;
          branch_of[g] = bmin;
          load[bmin] += gcost[g];
        }
      }
      if (hipEventRecord(ds->fork, s) != hipSuccess) return DF3C_E_HIP;
      for (int b = 0; b < NBRANCH - 1; ++b)
        if (hipStreamWaitEvent(ds->side[b], ds->fork, 0) != hipSuccess) return DF3C_E_HIP;
      for (int c : order) {
        const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
        const int br = branch_of[la * NLA + lb];
        hipStream_t bs = br == 0 ? s : ds->side[br - 1];
        JQArgs q{};
        q.a = base;
        q.orb_sorted = orb_sorted;
        q.aux_sorted = aux_sorted;
        q.Jall = Jc;
        q.seg = segd + p.cls_seg0[c];
        q.nseg = p.cls_seg0[c + 1] - p.cls_seg0[c];
        q.chunk = tt[c].chunk;
        q.total = p.cls_items[c];
        q.counter = ctr + c;
        const ClassInfo &ci = g_cls[lp][la][lb];
        q.a.nsub = class_nsub(c);
        const int64_t tpw = ci.tpwj / q.a.nsub;
        const int64_t need = (q.total + tpw * q.chunk - 1) / (tpw * q.chunk);
        const int grid = int(std::max<int64_t>(
            1, std::min<int64_t>(need, int64_t(ds->ncu) * tt[c].grid_per_cu)));
        if (timed(DF3C_KERNEL_JQ, c, bs, [&] { return ci.jq(q, grid, bs); }) != hipSuccess)
          return DF3C_E_HIP;
      }
      for (int b = 0; b < NBRANCH - 1; ++b)
        if (hipEventRecord(ds->join[b], ds->side[b]) != hipSuccess ||
            hipStreamWaitEvent(s, ds->join[b], 0) != hipSuccess)
          return DF3C_E_HIP;
    } else {
      for (int m = 0; m < nmol; ++m)
        for (int c : order) {
          const int lp = c / (NLA * NLA), la = (c / NLA) % NLA, lb = c % NLA;
          for (int g = p.cls_seg0[c]; g < p.cls_seg0[c + 1]; ++g) {
            const JSeg &sg = p.seg[g];
            if (sg.pad != m) continue;
            JArgs a = base;
            a.ash = orb_sorted + sg.ash;
            a.bsh = orb_sorted + sg.bsh;
            a.na = sg.na;
            a.nb = sg.nb;
            a.same = sg.same;
            a.psh = aux_sorted + sg.psh;
            a.arec = arec + int64_t(sg.psh) * AREC;
            a.np = sg.np;
            a.J = Jc + sg.jbase;
            a.nao = sg.nao;
            a.ao_base = sg.ao_base;
            a.npair = sg.npair;
            const ClassInfo &ci = g_cls[lp][la][lb];
            a.nsub = class_nsub(c);
            if (timed(DF3C_KERNEL_J, c, s, [&] {
                  return ci.jfn(a, grid_for(a.npair, ci.tpwj / a.nsub, ds->ncu), s);
                }) != hipSuccess)
              return DF3C_E_HIP;
          }
        }
    }
    if (orb->pure && p.np_max > 0) {
      const int gx = int(std::min<int64_t>((p.np_max * p.np_max + 255) / 256, 2048));
      hipLaunchKernelGGL(k_bra_pure_mol, dim3(gx, std::min(nmol, 65535)), dim3(256), 0, s, Jc,
                         pmol, nmol, prow, ao_off, orb->l, J, err);
      if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
    }
    return DF3C_OK;
  };

  if (!(flags & DF3C_GRAPH)) {
    if ((rc = enqueue())) return fail(rc);
    // the plan's host memory ends with this call: wait for its copies
    if ((flags & DF3C_ASYNC) && hipStreamSynchronize(s) != hipSuccess) return DF3C_E_HIP;
    return finish_call(flags, err, s);
  }
  // first call with DF3C_GRAPH: run once eagerly (sets kernel attributes), then
  // capture the same launches and keep the executable graph with its plan
  if ((rc = enqueue())) return fail(rc);
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(DF3C_E_HIP);
  rc = enqueue();
  if (hipStreamEndCapture(s, &graph) != hipSuccess || rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(rc ? rc : DF3C_E_HIP);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(DF3C_E_HIP);
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= GRAPH_CACHE) {
      // the oldest entry's graph and plan may still be in use by work queued
      // on any stream of the device: wait for the device first (rare)
      auto old = g_graphs.begin();
      for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
        if (it->second.stamp < old->second.stamp) old = it;
      if (hipDeviceSynchronize() != hipSuccess) return DF3C_E_HIP;
      (void)hipGraphExecDestroy(old->second.exec);
      g_graphs.erase(old);
    }
    GraphEntry &e = g_graphs[key];
    e.exec = exec;
    e.plan = pp;
    e.stamp = ++g_graph_clock;
  }
  return finish_call(flags, err, s);
}

}  // extern "C"
