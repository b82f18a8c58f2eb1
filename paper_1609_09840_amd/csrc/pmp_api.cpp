// Host side of libpmp: the C ABI declared in include/pmp.h.
//
// Argument checking, key tables, plan workspaces (one accumulator slot per
// 128-word block of buffer, zeroed once and kept zero by the kernel), grid
// sizing and the launches themselves. No hash arithmetic runs on the host.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <algorithm>
#include <vector>

#include "pmp.h"
#include "pmp_internal.h"

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PMP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// splitmix64 (Steele, Lea and Flood 2014): golden-gamma increment, then the
// mix64 finalizer.
uint64_t splitmix64(uint64_t* state) {
  uint64_t z = (*state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// largest admissible key a: p - kappa - 1 (Sec. 6.1, Table "parameters")
constexpr uint64_t AMAX32 = 4294967296ull - 14ull;  // 2^32 + 15 - 28 - 1
constexpr uint64_t AMAX64 = 0xfffffffffffffff4ull;  // 2^64 + 13 - 24 - 1 = 2^64 - 12

}  // namespace

namespace pmp {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace pmp

namespace pmp {
// the multiply-rate probe (pmp_probe.hip): `blocks` blocks of 256 threads
hipError_t launch_mad_probe(uint64_t* out, int blocks, uint32_t iters, hipStream_t s);
// the read-bandwidth probe: n16 pieces of 16 bytes
hipError_t launch_read_probe(const void* buf, uint64_t n16, uint32_t* out, int blocks, hipStream_t s);
}  // namespace pmp

struct pmp_plan {
  int device = 0;
  int32_t* status = nullptr;  // device
  pmp::Slot* slots = nullptr;  // device
  uint64_t nslots = 0;
  int g32 = 8, g64 = 8;
  uint32_t alpha = 768;        // per-string work in byte equivalents
  uint64_t wave_bytes = 8192;  // smallest share of work worth a wave
  int waves_per_cu = 0;        // 0: as many as stay resident
  int shares_per_wave = 1;     // shares of the work per wave (spread over the launch)
  int cus = 0;
  // descriptors of calls with more than two batches
  pmp::BatchArgs* desc_host = nullptr;  // pinned
  pmp::BatchArgs* desc_dev = nullptr;
  int desc_cap = 0;
  hipEvent_t desc_copied = nullptr;  // the last descriptor upload
  // captured graphs hold workspace pointers: while any exist, workspace that
  // grows is kept here instead of freed (freed with the last graph or the plan)
  int graphs = 0;
  std::vector<void*> retired;
  std::mutex mu;
};

namespace {

std::mutex g_default_mu;
std::map<std::pair<int, hipStream_t>, pmp_plan*> g_default;

int plan_init(pmp_plan* p, int device) {
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != device) return fail(PMP_E_INVALID_ARG, "plan device %d is not the current device %d", device, cur);
  p->device = device;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  p->cus = prop.multiProcessorCount;
  e = hipMalloc(&p->status, sizeof(int32_t));
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "workspace: %s", hipGetErrorString(e));
  e = hipMemset(p->status, 0, sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(e, "hipMemset");
  return PMP_OK;
}

// give up a workspace buffer that is being replaced
int plan_release(pmp_plan* p, void* ptr) {
  if (p->graphs > 0) {
    p->retired.push_back(ptr);
    return PMP_OK;
  }
  hipError_t e = hipFree(ptr);
  if (e != hipSuccess) return hip_fail(e, "hipFree");
  return PMP_OK;
}

// make room for n accumulator slots (zeroed)
int plan_slots(pmp_plan* p, uint64_t n) {
  if (n <= p->nslots) return PMP_OK;
  hipError_t e;
  if (p->slots) {
    int r = plan_release(p, p->slots);
    if (r) return r;
    p->slots = nullptr;
    p->nslots = 0;
  }
  const uint64_t want = n + n / 8 + 64;
  e = hipMalloc(&p->slots, want * sizeof(pmp::Slot));
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "workspace of %llu slots: %s", (unsigned long long)want,
                                   hipGetErrorString(e));
  e = hipMemset(p->slots, 0, want * sizeof(pmp::Slot));
  if (e != hipSuccess) return hip_fail(e, "hipMemset");
  p->nslots = want;
  return PMP_OK;
}

uint64_t slots_for(uint64_t buf_bytes, int wide) {
  const uint64_t blk = wide ? 1024 : 512;  // 128 words of 8 or 4 bytes
  return (buf_bytes + blk - 1) / blk + 2;
}

int default_plan(hipStream_t stream, pmp_plan** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_default_mu);
  auto key = std::make_pair(dev, stream);
  auto it = g_default.find(key);
  if (it != g_default.end()) {
    *out = it->second;
    return PMP_OK;
  }
  pmp_plan* p = new pmp_plan();
  int r = plan_init(p, dev);
  if (r != PMP_OK) {
    delete p;
    return r;
  }
  g_default[key] = p;
  *out = p;
  return PMP_OK;
}

int check_batch(const pmp_batch* b) {
  if (!b) return PMP_OK;
  if (b->count < 0) return fail(PMP_E_INVALID_ARG, "count %lld is negative", (long long)b->count);
  if (b->count == 0) return PMP_OK;
  if (!b->buf && b->buf_bytes) return fail(PMP_E_INVALID_ARG, "buf is NULL");
  if (!b->offsets || !b->keys || !b->out) return fail(PMP_E_INVALID_ARG, "offsets, keys and out must be non-NULL");
  if (b->flags & ~(PMP_NO_MIX | PMP_OUT_FIELD)) return fail(PMP_E_INVALID_ARG, "unknown flag bits 0x%x", b->flags);
  if (b->wide > 1) return fail(PMP_E_INVALID_ARG, "wide must be 0 or 1");
  const uint64_t W = b->wide ? 8 : 4;
  if (b->buf_bytes / W >= (1ull << 56) - 1)
    return fail(PMP_E_TOO_LONG, "a buffer of %llu bytes may hold strings of more than 2^56 words",
                (unsigned long long)b->buf_bytes);
  if (b->count > (int64_t)1 << 40) return fail(PMP_E_INVALID_ARG, "count too large");
  return PMP_OK;
}

int plan_desc(pmp_plan* p, int n) {
  if (n <= p->desc_cap) return PMP_OK;
  hipError_t e;
  if (p->desc_copied) {
    e = hipEventSynchronize(p->desc_copied);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  } else {
    e = hipEventCreateWithFlags(&p->desc_copied, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  }
  if (p->desc_host) (void)hipHostFree(p->desc_host);
  if (p->desc_dev) (void)hipFree(p->desc_dev);
  p->desc_host = nullptr;
  p->desc_dev = nullptr;
  p->desc_cap = 0;
  const int cap = n < 64 ? 64 : 2 * n;
  e = hipHostMalloc((void**)&p->desc_host, cap * sizeof(pmp::BatchArgs), hipHostMallocDefault);
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "descriptor staging: %s", hipGetErrorString(e));
  e = hipMalloc(&p->desc_dev, cap * sizeof(pmp::BatchArgs));
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "descriptor array: %s", hipGetErrorString(e));
  p->desc_cap = cap;
  return PMP_OK;
}

}  // namespace

namespace {

// A launch ready to go: kernel arguments (descriptor pointer still unset
// for more than two batches), grid and the batch descriptors.
struct Prepared {
  pmp::KArgs a;
  int grid = 0;
  int nb = 0;
  std::vector<pmp::BatchArgs> bv;
};

// Check the batches, size the plan workspace, fill the descriptors and pick
// the grid. Called with plan->mu held.
int prepare(pmp_plan* plan, const std::vector<const pmp_batch*>& list, Prepared& P) {
  using namespace pmp;
  const int nb = (int)list.size();
  P.nb = nb;
  std::memset(&P.a, 0, sizeof P.a);
  if (nb == 0) return PMP_OK;
  uint64_t need = 0;
  for (int k = 0; k < nb; ++k) need += slots_for(list[k]->buf_bytes, (int)list[k]->wide);
  int r = plan_slots(plan, need);
  if (r) return r;
  P.bv.assign(nb, BatchArgs{});
  uint64_t base = 0, work = 0;
  for (int k = 0; k < nb; ++k) {
    BatchArgs& B = P.bv[k];
    std::memset(&B, 0, sizeof B);
    B.buf = list[k]->buf;
    B.buf_bytes = list[k]->buf_bytes;
    B.offsets = list[k]->offsets;
    B.count = list[k]->count;
    B.keys = list[k]->keys;
    B.out = list[k]->out;
    B.flags = list[k]->flags;
    B.wide = list[k]->wide;
    B.slots = plan->slots + base;
    B.nslots = slots_for(list[k]->buf_bytes, (int)list[k]->wide);
    B.work0 = work;
    B.work = plan->alpha == PMP_ALPHA_BY_COUNT ? (uint64_t)list[k]->count
                                               : (uint64_t)plan->alpha * (uint64_t)list[k]->count + list[k]->buf_bytes;
    work += B.work;
    base += B.nslots;
  }
  if (nb <= 2)
    for (int k = 0; k < nb; ++k) P.a.b[k] = P.bv[k];
  P.a.batches = nullptr;
  P.a.nbatch = (uint32_t)nb;
  P.a.alpha = plan->alpha;
  P.a.status = plan->status;
  // one wave per `wave_bytes` of work, at most what the device keeps resident
  int per_cu = plan->waves_per_cu;
  if (per_cu <= 0) per_cu = 4 * batch_blocks_per_cu(plan->g32, plan->g64);
  if (per_cu <= 0) per_cu = 8;
  const uint64_t max_waves = (uint64_t)plan->cus * (uint64_t)per_cu;
  // (split by count: one wave per 64 strings at most)
  const bool by_count = plan->alpha == PMP_ALPHA_BY_COUNT;
  const uint64_t unit = by_count ? 64 : plan->wave_bytes;
  uint64_t waves = (work + unit - 1) / unit;
  if (waves < 1) waves = 1;
  if (waves > max_waves) waves = max_waves;
  P.a.total_waves = (uint32_t)waves;
  // small launches keep one share per wave
  uint64_t per_wave = (uint64_t)plan->shares_per_wave;
  while (per_wave > 1 && work / (waves * per_wave) < unit / 2) per_wave /= 2;
  P.a.per_wave = (uint32_t)per_wave;
  P.a.total = work;
  P.a.share = (work + waves * per_wave - 1) / (waves * per_wave);
  P.grid = (int)((waves + 3) / 4);
  return PMP_OK;
}

// Validate and keep the non-empty batches.
int collect(const pmp_batch* const* in, int n_in, std::vector<const pmp_batch*>& list) {
  if (n_in < 0) return fail(PMP_E_INVALID_ARG, "negative batch count");
  list.reserve(n_in);
  for (int k = 0; k < n_in; ++k) {
    int r = check_batch(in[k]);
    if (r) return r;
    if (in[k] && in[k]->count > 0) list.push_back(in[k]);
  }
  return PMP_OK;
}

int current_plan(pmp_plan** plan, hipStream_t stream) {
  if (!*plan) {
    int r = default_plan(stream, plan);
    if (r) return r;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != (*plan)->device)
    return fail(PMP_E_INVALID_ARG, "plan belongs to device %d, current is %d", (*plan)->device, dev);
  return PMP_OK;
}

}  // namespace

namespace pmp {

int32_t* plan_status_word(pmp_plan* plan) { return plan ? plan->status : nullptr; }

int plan_clear_async(pmp_plan* plan, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(plan->mu);
  hipError_t e = hipMemsetAsync(plan->status, 0, sizeof(int32_t), stream);
  if (e == hipSuccess && plan->slots) e = hipMemsetAsync(plan->slots, 0, plan->nslots * sizeof(Slot), stream);
  return e == hipSuccess ? PMP_OK : hip_fail(e, "hipMemsetAsync");
}

// Up to two batches in one launch with workspace the caller brings: `slots`
// node accumulators (nslots of them, zero on entry, left zero by a launch
// whose offsets are in order) and the status word; `cus` and `per_cu` size
// the grid. Nothing is allocated: the plan below lives on the stack and
// only describes that workspace, with the default tiles and work weight.
int run_static(const pmp_batch* const* in, int n_in, Slot* slots, uint64_t nslots, int32_t* status, int cus,
               hipStream_t stream) {
  std::vector<const pmp_batch*> list;
  int r = collect(in, n_in, list);
  if (r || list.empty()) return r;
  uint64_t need = 0;
  for (const pmp_batch* b : list) need += slots_for(b->buf_bytes, (int)b->wide);
  if (need > nslots)
    return fail(PMP_E_NOMEM, "the batches need %llu node accumulators (16 bytes each); the static scratch holds %llu",
                (unsigned long long)need, (unsigned long long)nslots);
  pmp_plan plan;  // no device memory of its own
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  plan.device = dev;
  plan.cus = cus;
  plan.slots = slots;
  plan.nslots = nslots;
  plan.status = status;
  Prepared P;
  r = prepare(&plan, list, P);  // need <= nslots: the workspace is not grown
  if (r) return r;
  e = launch_batch(P.a, P.grid, plan.g32, plan.g64, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return PMP_OK;
}

// Hash n batches in one launch.
int run_batches(pmp_plan* plan, const pmp_batch* const* in, int n_in, hipStream_t stream) {
  std::vector<const pmp_batch*> list;
  int r = collect(in, n_in, list);
  if (r || list.empty()) return r;
  r = current_plan(&plan, stream);
  if (r) return r;
  std::lock_guard<std::mutex> lk(plan->mu);
  Prepared P;
  r = prepare(plan, list, P);
  if (r) return r;
  hipError_t e;
  if (P.nb > 2) {
    r = plan_desc(plan, P.nb);
    if (r) return r;
    // the staging buffer may still feed the previous upload
    e = hipEventSynchronize(plan->desc_copied);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    std::memcpy(plan->desc_host, P.bv.data(), P.nb * sizeof(BatchArgs));
    e = hipMemcpyAsync(plan->desc_dev, plan->desc_host, P.nb * sizeof(BatchArgs), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(plan->desc_copied, stream);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    P.a.batches = plan->desc_dev;
  }
  e = launch_batch(P.a, P.grid, plan->g32, plan->g64, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return PMP_OK;
}

}  // namespace pmp

// A captured launch (hipGraph) over fixed batch descriptors.
struct pmp_graph {
  pmp_plan* plan = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  pmp::BatchArgs* desc = nullptr;  // device, owned (more than two batches)
};

namespace {

int run_two(pmp_plan* plan, const pmp_batch* b0, const pmp_batch* b1, hipStream_t stream) {
  const pmp_batch* l[2] = {b0, b1};
  return pmp::run_batches(plan, l, 2, stream);
}

}  // namespace

extern "C" {

const char* pmp_last_error(void) { return g_err.c_str(); }
const char* pmp_version(void) { return "pmp 0.1 (gfx950)"; }

int pmp_expand_keys32(uint64_t seed, uint32_t* keys_out) {
  if (!keys_out) return fail(PMP_E_INVALID_ARG, "keys_out is NULL");
  uint64_t s = seed;
  for (int i = 0; i < PMP_LEVELS * PMP_BLOCK; ++i) {
    uint64_t c;
    do {
      c = splitmix64(&s) >> 32;
    } while (c < 1 || c > AMAX32);
    keys_out[i] = (uint32_t)c;
  }
  for (int j = 0; j < PMP_LEVELS; ++j) keys_out[PMP_LEVELS * PMP_BLOCK + j] = (uint32_t)(splitmix64(&s) >> 32);
  return PMP_OK;
}

int pmp_expand_keys64(uint64_t seed, uint64_t* keys_out) {
  if (!keys_out) return fail(PMP_E_INVALID_ARG, "keys_out is NULL");
  uint64_t s = seed;
  for (int i = 0; i < PMP_LEVELS * PMP_BLOCK; ++i) {
    uint64_t c;
    do {
      c = splitmix64(&s);
    } while (c < 1 || c > AMAX64);
    keys_out[i] = c;
  }
  for (int j = 0; j < PMP_LEVELS; ++j) keys_out[PMP_LEVELS * PMP_BLOCK + j] = splitmix64(&s);
  return PMP_OK;
}

int pmp_check_keys32(const uint32_t* keys) {
  if (!keys) return fail(PMP_E_INVALID_ARG, "keys is NULL");
  for (int i = 0; i < PMP_LEVELS * PMP_BLOCK; ++i)
    if (keys[i] > AMAX32) return fail(PMP_E_KEY_RANGE, "key a[%d][%d] = %u exceeds 2^32 - 14", i / PMP_BLOCK,
                                      i % PMP_BLOCK, keys[i]);
  return PMP_OK;
}

int pmp_check_keys64(const uint64_t* keys) {
  if (!keys) return fail(PMP_E_INVALID_ARG, "keys is NULL");
  for (int i = 0; i < PMP_LEVELS * PMP_BLOCK; ++i)
    if (keys[i] > AMAX64)
      return fail(PMP_E_KEY_RANGE, "key a[%d][%d] = %llu exceeds 2^64 - 12", i / PMP_BLOCK, i % PMP_BLOCK,
                  (unsigned long long)keys[i]);
  return PMP_OK;
}

int pmp_plan_create(int device, pmp_plan** plan_out) {
  if (!plan_out) return fail(PMP_E_INVALID_ARG, "plan_out is NULL");
  pmp_plan* p = new pmp_plan();
  int r = plan_init(p, device);
  if (r) {
    delete p;
    return r;
  }
  *plan_out = p;
  return PMP_OK;
}

int pmp_plan_destroy(pmp_plan* plan) {
  if (!plan) return PMP_OK;
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    for (auto it = g_default.begin(); it != g_default.end(); ++it)
      if (it->second == plan) return fail(PMP_E_INVALID_ARG, "default plans are owned by the library");
  }
  (void)hipDeviceSynchronize();
  if (plan->slots) (void)hipFree(plan->slots);
  if (plan->status) (void)hipFree(plan->status);
  if (plan->desc_host) (void)hipHostFree(plan->desc_host);
  if (plan->desc_dev) (void)hipFree(plan->desc_dev);
  if (plan->desc_copied) (void)hipEventDestroy(plan->desc_copied);
  for (void* q : plan->retired) (void)hipFree(q);
  delete plan;
  return PMP_OK;
}

int pmp_plan_reserve(pmp_plan* plan, uint64_t max_buf_bytes, int64_t max_count) {
  if (!plan || max_count < 0) return fail(PMP_E_INVALID_ARG, "bad plan or count");
  std::lock_guard<std::mutex> lk(plan->mu);
  // PM+32 blocks are the smaller ones, so they bound either variant; a mixed
  // call needs at most two batches' worth of padding slots
  return plan_slots(plan, slots_for(max_buf_bytes, 0) + 2);
}

int pmp_plan_status(pmp_plan* plan, pmp_stream_t stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!plan) {
    int r = default_plan(s, &plan);
    if (r) return r;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  std::lock_guard<std::mutex> lk(plan->mu);
  int32_t st = 0;
  e = hipMemcpy(&st, plan->status, sizeof st, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  if (!st) return PMP_OK;
  // a bad batch can leave node accumulators half filled: clear everything
  e = hipMemset(plan->status, 0, sizeof(int32_t));
  if (e == hipSuccess && plan->slots) e = hipMemset(plan->slots, 0, plan->nslots * sizeof(pmp::Slot));
  if (e != hipSuccess) return hip_fail(e, "hipMemset");
  if (st & pmp::STATUS_OFFSETS)
    return fail(PMP_E_OFFSETS, "offsets out of order or past buf_bytes (or a string over 2^56 words)");
  return fail(PMP_E_INTERNAL, "a tree node fell outside the workspace");
}

int pmp_plan_set_tile(pmp_plan* plan, int wide, int lanes_per_block) {
  if (!plan) return fail(PMP_E_INVALID_ARG, "plan is NULL");
  std::lock_guard<std::mutex> lk(plan->mu);
  const int g32 = wide ? plan->g32 : (lanes_per_block ? lanes_per_block : 8);
  const int g64 = wide ? (lanes_per_block ? lanes_per_block : 16) : plan->g64;
  if (!pmp::batch_tiles_supported(g32, g64))
    return fail(PMP_E_INVALID_ARG, "no kernel for %d (PM+32) and %d (PM+64) lanes per block", g32, g64);
  plan->g32 = g32;
  plan->g64 = g64;
  return PMP_OK;
}

int pmp_plan_tune(pmp_plan* plan, int waves_per_cu, uint32_t alpha, uint64_t wave_bytes, int shares_per_wave) {
  if (!plan || waves_per_cu < 0 || waves_per_cu > 64 || shares_per_wave < 0 || shares_per_wave > 64)
    return fail(PMP_E_INVALID_ARG, "bad tuning values");
  std::lock_guard<std::mutex> lk(plan->mu);
  plan->waves_per_cu = waves_per_cu;
  if (alpha) plan->alpha = alpha;
  if (wave_bytes) plan->wave_bytes = wave_bytes;
  if (shares_per_wave) plan->shares_per_wave = shares_per_wave;
  return PMP_OK;
}

int pmp_hash32(pmp_plan* plan, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets, int64_t count,
               const uint32_t* d_keys, void* d_out, uint32_t flags, pmp_stream_t stream) {
  pmp_batch b{d_buf, buf_bytes, d_offsets, count, d_keys, d_out, flags, 0};
  return run_two(plan, &b, nullptr, (hipStream_t)stream);
}

int pmp_hash64(pmp_plan* plan, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets, int64_t count,
               const uint64_t* d_keys, void* d_out, uint32_t flags, pmp_stream_t stream) {
  pmp_batch b{d_buf, buf_bytes, d_offsets, count, d_keys, d_out, flags, 1};
  return run_two(plan, &b, nullptr, (hipStream_t)stream);
}

int pmp_hash_mixed(pmp_plan* plan, const pmp_batch* b0, const pmp_batch* b1, pmp_stream_t stream) {
  return run_two(plan, b0, b1, (hipStream_t)stream);
}

int pmp_hash_many(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_stream_t stream) {
  if (nbatch < 0 || (nbatch > 0 && !batches)) return fail(PMP_E_INVALID_ARG, "bad batch array");
  std::vector<const pmp_batch*> l(nbatch);
  for (int k = 0; k < nbatch; ++k) l[k] = batches + k;
  return pmp::run_batches(plan, l.data(), nbatch, (hipStream_t)stream);
}

int pmp_graph_create(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_graph** out) {
  if (!plan || !out || nbatch < 0 || (nbatch > 0 && !batches)) return fail(PMP_E_INVALID_ARG, "bad arguments");
  *out = nullptr;
  std::vector<const pmp_batch*> in(nbatch);
  for (int k = 0; k < nbatch; ++k) in[k] = batches + k;
  std::vector<const pmp_batch*> list;
  int r = collect(in.data(), nbatch, list);
  if (r) return r;
  r = current_plan(&plan, nullptr);
  if (r) return r;
  std::lock_guard<std::mutex> lk(plan->mu);
  Prepared P;
  r = prepare(plan, list, P);  // grows the workspace now, outside the capture
  if (r) return r;
  pmp_graph* g = new pmp_graph();
  g->plan = plan;
  hipError_t e = hipSuccess;
  hipStream_t cs = nullptr;
  auto bail = [&](int code, const char* what) {
    if (cs) (void)hipStreamDestroy(cs);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->desc) (void)hipFree(g->desc);
    delete g;
    return code == PMP_E_HIP ? hip_fail(e, what) : fail(code, "%s: %s", what, hipGetErrorString(e));
  };
  if (P.nb > 2) {
    e = hipMalloc(&g->desc, P.nb * sizeof(pmp::BatchArgs));
    if (e != hipSuccess) return bail(PMP_E_NOMEM, "graph descriptors");
    e = hipMemcpy(g->desc, P.bv.data(), P.nb * sizeof(pmp::BatchArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(PMP_E_HIP, "graph descriptor upload");
    P.a.batches = g->desc;
  }
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(PMP_E_HIP, "capture stream");
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bail(PMP_E_HIP, "hipStreamBeginCapture");
  hipError_t le = P.nb ? pmp::launch_batch(P.a, P.grid, plan->g32, plan->g64, cs) : hipSuccess;
  e = hipStreamEndCapture(cs, &g->graph);
  if (le != hipSuccess) {
    e = le;
    return bail(PMP_E_HIP, "captured launch");
  }
  if (e != hipSuccess) return bail(PMP_E_HIP, "hipStreamEndCapture");
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(PMP_E_HIP, "hipGraphInstantiate");
  (void)hipStreamDestroy(cs);
  ++plan->graphs;
  *out = g;
  return PMP_OK;
}

int pmp_graph_launch(pmp_graph* graph, pmp_stream_t stream) {
  if (!graph) return fail(PMP_E_INVALID_ARG, "graph is NULL");
  hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return PMP_OK;
}

int pmp_graph_destroy(pmp_graph* graph) {
  if (!graph) return PMP_OK;
  (void)hipDeviceSynchronize();  // replays may still read the descriptors
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  if (graph->desc) (void)hipFree(graph->desc);
  {
    std::lock_guard<std::mutex> lk(graph->plan->mu);
    if (--graph->plan->graphs == 0) {
      for (void* q : graph->plan->retired) (void)hipFree(q);
      graph->plan->retired.clear();
    }
  }
  delete graph;
  return PMP_OK;
}

int pmp_plan_autotune(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_stream_t stream,
                      pmp_tuning* best) {
  if (!plan || nbatch < 0 || (nbatch > 0 && !batches)) return fail(PMP_E_INVALID_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  // time one configuration: one warm launch, then the mean of `reps`
  auto measure = [&](float* ms, int reps) -> int {
    int r = pmp_hash_many(plan, batches, nbatch, stream);
    if (r) return r;
    hipError_t x = hipEventRecord(e0, s);
    for (int k = 0; k < reps && !r; ++k) r = pmp_hash_many(plan, batches, nbatch, stream);
    if (r) return r;
    if (x == hipSuccess) x = hipEventRecord(e1, s);
    if (x == hipSuccess) x = hipEventSynchronize(e1);
    if (x == hipSuccess) x = hipEventElapsedTime(ms, e0, e1);
    if (x != hipSuccess) return hip_fail(x, "autotune timing");
    *ms /= reps;
    return PMP_OK;
  };
  pmp_tuning cur{plan->g32, plan->g64, plan->alpha, plan->waves_per_cu, plan->shares_per_wave, 0.f};
  pmp_tuning top = cur;
  top.ms = 1e30f;
  auto apply = [&](const pmp_tuning& t) {
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->g32 = t.g32;
    plan->g64 = t.g64;
    plan->alpha = t.alpha;
    plan->waves_per_cu = t.waves_per_cu;
    plan->shares_per_wave = t.shares_per_wave;
  };
  std::vector<pmp_tuning> seen;  // every setting tried, with its time
  auto trial = [&](pmp_tuning t) -> int {
    apply(t);
    float ms = 0;
    const int rr = measure(&ms, 3);
    if (!rr) {
      t.ms = ms;
      seen.push_back(t);
      if (ms < top.ms) top = t;
    }
    return rr;
  };
  int pairs[16][2];
  const int np = pmp::batch_tile_pairs(pairs, 16);
  const uint32_t alphas[] = {256, 512, 768, 1024, 1536, 2048, PMP_ALPHA_BY_COUNT};
  int r = PMP_OK;
  for (int t = 0; t < np && !r; ++t)
    for (uint32_t al : alphas)
      if (!r) r = trial(pmp_tuning{pairs[t][0], pairs[t][1], al, 0, 1, 0.f});
  const int shares[] = {2, 4};
  for (int sp : shares)
    if (!r) r = trial(pmp_tuning{top.g32, top.g64, top.alpha, 0, sp, 0.f});
  const int wpcs[] = {4, 12, 16};
  for (int wv : wpcs)
    if (!r) r = trial(pmp_tuning{top.g32, top.g64, top.alpha, wv, top.shares_per_wave, 0.f});
  // the four fastest settings timed again over ten launches each: short
  // timings of settings within a few percent of each other are noisy
  if (!r && seen.size() > 1) {
    std::sort(seen.begin(), seen.end(), [](const pmp_tuning& a, const pmp_tuning& b) { return a.ms < b.ms; });
    top.ms = 1e30f;
    for (size_t k = 0; k < seen.size() && k < 4 && !r; ++k) {
      pmp_tuning t = seen[k];
      apply(t);
      float ms = 0;
      r = measure(&ms, 10);
      if (!r && ms < top.ms) {
        t.ms = ms;
        top = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const pmp_tuning keep = r ? cur : top;
  apply(keep);
  if (best) *best = keep;
  return r;
}

int pmp_hash_plain(int wide, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* h_offsets, int64_t count,
                   const void* d_keys, void* d_out, uint32_t flags, void* d_scratch, uint64_t scratch_bytes,
                   pmp_stream_t stream) {
  if (count < 0 || (count > 0 && (!h_offsets || !d_keys || !d_out || !d_scratch)))
    return fail(PMP_E_INVALID_ARG, "bad arguments");
  if (flags & ~(PMP_NO_MIX | PMP_OUT_FIELD)) return fail(PMP_E_INVALID_ARG, "unknown flag bits");
  for (int64_t i = 0; i < count; ++i) {
    const int64_t o0 = h_offsets[i], o1 = h_offsets[i + 1];
    if (o0 < 0 || o1 < o0 || (uint64_t)o1 > buf_bytes)
      return fail(PMP_E_OFFSETS, "string %lld: offsets [%lld, %lld) outside [0, %llu]", (long long)i, (long long)o0,
                  (long long)o1, (unsigned long long)buf_bytes);
    hipError_t e = pmp::launch_plain_string(wide, d_buf, buf_bytes, o0, o1 - o0, d_keys, d_out, i, flags,
                                            (uint4*)d_scratch, scratch_bytes / 16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plain launch (scratch too small?)");
  }
  return PMP_OK;
}

int pmp_debug_fold(int wide, const void* d_w0, const void* d_w1, const uint32_t* d_w2, void* d_z, int64_t n,
                   pmp_stream_t stream) {
  if (n < 0 || (n > 0 && (!d_w0 || !d_w1 || !d_w2 || !d_z))) return fail(PMP_E_INVALID_ARG, "bad arguments");
  if (n == 0) return PMP_OK;
  hipError_t e = pmp::launch_debug_fold(wide, d_w0, d_w1, d_w2, d_z, n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "fold launch");
  return PMP_OK;
}

int pmp_probe_mad_rate(double* mads_per_s) {
  if (!mads_per_s) return fail(PMP_E_INVALID_ARG, "mads_per_s is NULL");
  *mads_per_s = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "device properties");
  const int blocks = prop.multiProcessorCount * 8;  // 8 waves per SIMD's worth of lanes
  const uint32_t iters = 4096;
  uint64_t* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "probe buffer: %s", hipGetErrorString(e));
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0;
  if (e == hipSuccess) e = pmp::launch_mad_probe(out, blocks, iters, s);  // warm
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = pmp::launch_mad_probe(out, blocks, iters, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e1) (void)hipEventDestroy(e1);
  if (e0) (void)hipEventDestroy(e0);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "mad probe");
  if (ms <= 0) return fail(PMP_E_HIP, "mad probe took no time");
  *mads_per_s = 3.0 * blocks * 256.0 * iters * 8.0 / (ms * 1e-3);
  return PMP_OK;
}

int pmp_probe_read_bw(const void* d_buf, uint64_t bytes, double* bytes_per_s) {
  if (!bytes_per_s || !d_buf) return fail(PMP_E_INVALID_ARG, "NULL argument");
  *bytes_per_s = 0;
  if (bytes < (1u << 20) || ((uintptr_t)d_buf & 15u)) return fail(PMP_E_INVALID_ARG, "need >= 1 MiB, 16-byte aligned");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "device properties");
  const int blocks = prop.multiProcessorCount * 16;  // 16 waves per SIMD's worth of lanes
  const uint64_t n16 = bytes / 16;
  uint32_t* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint32_t));
  if (e != hipSuccess) return fail(PMP_E_NOMEM, "probe buffer: %s", hipGetErrorString(e));
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0;
  const int reps = 5;
  if (e == hipSuccess) e = pmp::launch_read_probe(d_buf, n16, out, blocks, s);  // warm
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = pmp::launch_read_probe(d_buf, n16, out, blocks, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e1) (void)hipEventDestroy(e1);
  if (e0) (void)hipEventDestroy(e0);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "read probe");
  if (ms <= 0) return fail(PMP_E_HIP, "read probe took no time");
  *bytes_per_s = (double)reps * (double)(n16 * 16) / (ms * 1e-3);
  return PMP_OK;
}

// ---------------------------------------------------------------------------
// PM+128 over p = 2^128 + 51.
int pmp_expand_keys128(uint64_t seed, uint64_t* keys_out) {
  if (!keys_out) return fail(PMP_E_INVALID_ARG, "keys_out is NULL");
  uint64_t st = seed;
  for (int i = 0; i < PMP_KEYS; ++i) {
    for (;;) {
      const uint64_t lo = splitmix64(&st), hi = splitmix64(&st);
      keys_out[2 * i] = lo;
      keys_out[2 * i + 1] = hi;
      if (i >= PMP_LEVELS * PMP_BLOCK) break;  // b: any 128-bit value
      // a in [1, 2^128 - 50]
      if ((lo | hi) != 0 && !(hi == ~0ull && lo > ~0ull - 49)) break;
    }
  }
  return PMP_OK;
}

int pmp_check_keys128(const uint64_t* keys) {
  if (!keys) return fail(PMP_E_INVALID_ARG, "keys is NULL");
  for (int i = 0; i < PMP_LEVELS * PMP_BLOCK; ++i) {
    const uint64_t lo = keys[2 * i], hi = keys[2 * i + 1];
    if (hi == ~0ull && lo > ~0ull - 49) return fail(PMP_E_KEY_RANGE, "key %d above 2^128 - 50", i);
  }
  return PMP_OK;
}

uint64_t pmp_hash128_scratch_bytes(int64_t count, uint64_t buf_bytes) {
  return count < 0 ? 0 : pmp::pm128_scratch_bytes(count, buf_bytes);
}

int pmp_hash128(const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets, int64_t count,
                const uint64_t* d_keys, void* d_out, uint32_t flags, void* d_scratch, uint64_t scratch_bytes,
                pmp_stream_t stream) {
  if (count < 0 || count > ((int64_t)1 << 40)) return fail(PMP_E_INVALID_ARG, "bad count");
  if (count == 0) return PMP_OK;
  if (!d_offsets || !d_keys || !d_out || !d_scratch || (!d_buf && buf_bytes))
    return fail(PMP_E_INVALID_ARG, "NULL argument");
  if (flags & ~(PMP_NO_MIX | PMP_OUT_FIELD)) return fail(PMP_E_INVALID_ARG, "unknown flag bits");
  if (buf_bytes / 16 >= (1ull << 56) - 1) return fail(PMP_E_TOO_LONG, "buffer too long for 8 levels");
  if (scratch_bytes < pmp::pm128_scratch_bytes(count, buf_bytes))
    return fail(PMP_E_INVALID_ARG, "d_scratch holds %llu bytes, %llu needed", (unsigned long long)scratch_bytes,
                (unsigned long long)pmp::pm128_scratch_bytes(count, buf_bytes));
  hipError_t e = pmp::launch_pm128(d_buf, buf_bytes, d_offsets, count, d_keys, d_out, flags, d_scratch,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "PM+128 launch");
  return PMP_OK;
}

// ---------------------------------------------------------------------------
// Hash table of variable-length keys: the batch kernel hashes, the table
// kernels bucket and probe.
uint64_t pmp_table_work_bytes(uint64_t nbuckets) { return pmp::table_work_bytes(nbuckets); }

int pmp_table_build(pmp_plan* plan, const pmp_batch* keys, uint64_t nbuckets, int64_t* d_bucket_start,
                    pmp_table_entry* d_entries, void* d_work, uint64_t work_bytes, pmp_stream_t stream) {
  if (!keys || !d_bucket_start || !d_work || (keys->count > 0 && !d_entries))
    return fail(PMP_E_INVALID_ARG, "NULL argument");
  int r = check_batch(keys);
  if (r) return r;
  if (keys->flags & PMP_OUT_FIELD) return fail(PMP_E_INVALID_ARG, "a table keys on n-bit outputs (no PMP_OUT_FIELD)");
  if (nbuckets < 1 || nbuckets > (1ull << 31)) return fail(PMP_E_INVALID_ARG, "nbuckets must be in [1, 2^31]");
  if (work_bytes < pmp::table_work_bytes(nbuckets))
    return fail(PMP_E_INVALID_ARG, "d_work holds %llu bytes, %llu needed", (unsigned long long)work_bytes,
                (unsigned long long)pmp::table_work_bytes(nbuckets));
  if (keys->count > 0) {
    r = run_two(plan, keys, nullptr, (hipStream_t)stream);
    if (r) return r;
  }
  hipError_t e = pmp::launch_table_build(keys->out, keys->wide, keys->count, nbuckets, keys->offsets,
                                         d_bucket_start, d_entries, d_work, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "table build launch");
  return PMP_OK;
}

int pmp_table_probe(pmp_plan* plan, const pmp_batch* queries, const pmp_batch* keys, uint64_t nbuckets,
                    const int64_t* d_bucket_start, const pmp_table_entry* d_entries, int64_t* d_result,
                    pmp_stream_t stream) {
  if (!queries || !keys || !d_bucket_start || (queries->count > 0 && !d_result))
    return fail(PMP_E_INVALID_ARG, "NULL argument");
  int r = check_batch(queries);
  if (r) return r;
  r = check_batch(keys);
  if (r) return r;
  if (queries->wide != keys->wide || queries->keys != keys->keys || queries->flags != keys->flags)
    return fail(PMP_E_INVALID_ARG, "queries and keys must share the variant, the key table and the flags");
  if (keys->flags & PMP_OUT_FIELD) return fail(PMP_E_INVALID_ARG, "a table keys on n-bit outputs (no PMP_OUT_FIELD)");
  if (nbuckets < 1 || nbuckets > (1ull << 31)) return fail(PMP_E_INVALID_ARG, "nbuckets must be in [1, 2^31]");
  if (queries->count == 0) return PMP_OK;
  r = run_two(plan, queries, nullptr, (hipStream_t)stream);
  if (r) return r;
  hipError_t e = pmp::launch_table_probe(queries->buf, queries->offsets, queries->count, queries->out, keys->buf,
                                         keys->wide, nbuckets, d_bucket_start, d_entries, d_result,
                                         (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "table probe launch");
  return PMP_OK;
}

// ---------------------------------------------------------------------------
// Incremental hashing: the host keeps the byte count, from which every count
// the kernels need follows (blocks completed, nodes per level, carried bytes).
}  // extern "C"

struct pmp_incr {
  int wide = 0;
  const void* keys = nullptr;
  hipStream_t stream = nullptr;
  pmp::IncrState* st = nullptr;  // device state, followed by two sets of boundary sums
  uint64_t* sums = nullptr;
  uint4* z = nullptr;            // per parity two level-output buffers of cap entries,
                                 // then cap node accumulators
  uint64_t cap = 0;
  uint64_t len = 0;              // bytes appended since creation or reset
  int parity = 0;                // buffers of the next append that completes blocks
  bool pending = false;          // the last such append's tree step has not run yet
  uint64_t p_s1 = 0, p_k = 0;    // that append's blocks
};

namespace {

// workspace entries for an append of n bytes: the level-2 nodes it can touch
// (n / (128 W * 128) + 2) and two more
uint64_t incr_nodes_for(const pmp_incr* h, uint64_t n) {
  const uint64_t C = (uint64_t)PMP_BLOCK * (h->wide ? 8 : 4);
  return n / (C * PMP_BLOCK) + 4;
}

size_t incr_workspace_bytes(uint64_t entries) {
  return entries * (4 * sizeof(uint4) + sizeof(pmp::Slot));
}

// the tree step left by the last append that completed blocks
pmp::IncrTree incr_prev(const pmp_incr* h) {
  const int q = h->parity ^ 1;
  return pmp::IncrTree{h->p_s1, h->p_k, h->z + 2 * q * h->cap, h->z + (2 * q + 1) * h->cap, h->sums + 8 * q};
}

int incr_grow(pmp_incr* h, uint64_t entries) {
  if (entries <= h->cap) return PMP_OK;
  hipError_t e;
  if (h->pending) {  // the pending tree step reads the old buffers
    e = pmp::launch_incr_flush(h->wide, h->st, h->keys, incr_prev(h), h->stream);
    if (e != hipSuccess) return hip_fail(e, "tree step launch");
    h->pending = false;
  }
  // queued appends may still use the old buffers
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (h->z) {
    e = hipFree(h->z);
    h->z = nullptr;
    h->cap = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  const size_t bytes = incr_workspace_bytes(entries);
  e = hipMalloc((void**)&h->z, bytes);
  if (e != hipSuccess) {
    h->z = nullptr;
    return fail(PMP_E_NOMEM, "incremental workspace of %llu bytes: %s", (unsigned long long)bytes,
                hipGetErrorString(e));
  }
  // the node accumulators start at zero and the kernels return them to zero
  e = hipMemset(h->z, 0, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMemset");
  h->cap = entries;
  return PMP_OK;
}

}  // namespace

extern "C" {

int pmp_incr_create(int wide, const void* d_keys, pmp_stream_t stream, pmp_incr** out) {
  if (!out) return fail(PMP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d_keys) return fail(PMP_E_INVALID_ARG, "d_keys is NULL");
  if (wide != 0 && wide != 1) return fail(PMP_E_INVALID_ARG, "wide must be 0 (PM+32) or 1 (PM+64)");
  pmp_incr* h = new pmp_incr;
  h->wide = wide;
  h->keys = d_keys;
  h->stream = (hipStream_t)stream;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, sizeof(pmp::IncrState) + 16 * sizeof(uint64_t));
  if (e != hipSuccess) {
    delete h;
    return fail(PMP_E_NOMEM, "incremental state: %s", hipGetErrorString(e));
  }
  h->st = (pmp::IncrState*)mem;
  h->sums = (uint64_t*)((char*)mem + sizeof(pmp::IncrState));
  int r = incr_grow(h, incr_nodes_for(h, 0));
  if (r == PMP_OK) {
    e = pmp::launch_incr_reset(h->st, h->stream);
    if (e != hipSuccess) r = hip_fail(e, "state reset");
  }
  if (r != PMP_OK) {
    (void)hipFree(h->z);
    (void)hipFree(h->st);
    delete h;
    return r;
  }
  *out = h;
  return PMP_OK;
}

int pmp_incr_reserve(pmp_incr* h, uint64_t max_piece_bytes) {
  if (!h) return fail(PMP_E_INVALID_ARG, "handle is NULL");
  return incr_grow(h, incr_nodes_for(h, max_piece_bytes));
}

int pmp_incr_append(pmp_incr* h, const uint8_t* d_piece, uint64_t nbytes) {
  if (!h) return fail(PMP_E_INVALID_ARG, "handle is NULL");
  if (nbytes == 0) return PMP_OK;
  if (!d_piece) return fail(PMP_E_INVALID_ARG, "d_piece is NULL");
  const uint64_t C = (uint64_t)PMP_BLOCK * (h->wide ? 8 : 4);
  // the padded string may have at most 128^8 words: 128^7 blocks
  const uint64_t max_blocks = 1ull << 49;
  if (nbytes > (1ull << 62) || h->len + nbytes < h->len || (h->len + nbytes) / C + 1 > max_blocks)
    return fail(PMP_E_TOO_LONG, "the string would need more than %d levels", PMP_LEVELS);
  if (nbytes / (C * pmp::INCR_SEG) + 2 > 0x7fffffffull)
    return fail(PMP_E_INVALID_ARG, "piece of %llu bytes: append it in smaller pieces", (unsigned long long)nbytes);
  const uint64_t len1 = h->len + nbytes;
  const uint64_t s1 = h->len / C, k = len1 / C - s1;
  const uint32_t t = (uint32_t)(h->len % C);
  hipError_t e;
  if (k == 0) {
    e = pmp::launch_incr_carry(h->st, t, d_piece, (int64_t)nbytes, h->stream);
    if (e != hipSuccess) return hip_fail(e, "carry launch");
  } else {
    const uint64_t nwg = (s1 + k - 1) / pmp::INCR_SEG - s1 / pmp::INCR_SEG + 1;
    const uint64_t nodes = (s1 + k - 1) / PMP_BLOCK - s1 / PMP_BLOCK + 1;
    int r = incr_grow(h, nodes + 2);
    if (r != PMP_OK) return r;
    pmp::IncrArgs a{};
    a.piece = d_piece;
    a.n = (int64_t)nbytes;
    a.s1 = s1;
    a.k = k;
    a.t = t;
    a.r_new = (uint32_t)(len1 % C);
    a.nwg = (uint32_t)nwg;
    a.keys = h->keys;
    a.st = h->st;
    const int q = h->parity;
    a.za = h->z + 2 * q * h->cap;
    a.zb = h->z + (2 * q + 1) * h->cap;
    a.slots = (pmp::Slot*)(h->z + 4 * h->cap);
    a.sums = h->sums + 8 * q;
    a.pending = h->pending ? 1u : 0u;
    a.prev = incr_prev(h);
    e = pmp::launch_incr_append(h->wide, a, h->stream);
    if (e != hipSuccess) return hip_fail(e, "append launch");
    h->pending = true;
    h->p_s1 = s1;
    h->p_k = k;
    h->parity ^= 1;
  }
  h->len = len1;
  return PMP_OK;
}

int pmp_incr_digest(pmp_incr* h, void* d_out, uint32_t flags) {
  if (!h) return fail(PMP_E_INVALID_ARG, "handle is NULL");
  if (!d_out) return fail(PMP_E_INVALID_ARG, "d_out is NULL");
  if (flags & ~(PMP_NO_MIX | PMP_OUT_FIELD)) return fail(PMP_E_INVALID_ARG, "unknown flag bits");
  const uint64_t C = (uint64_t)PMP_BLOCK * (h->wide ? 8 : 4);
  uint64_t nodes[PMP_LEVELS + 1] = {0};
  nodes[1] = h->len / C + 1;  // the open block holds at least the pad word
  for (int j = 2; j <= PMP_LEVELS; ++j) nodes[j] = (nodes[j - 1] + PMP_BLOCK - 1) / PMP_BLOCK;
  hipError_t e = pmp::launch_incr_digest(h->wide, h->st, (uint32_t)(h->len % C), nodes, h->keys, d_out, flags,
                                         h->pending ? 1u : 0u, incr_prev(h), h->stream);
  if (e != hipSuccess) return hip_fail(e, "digest launch");
  h->pending = false;  // the digest ran it
  return PMP_OK;
}

int pmp_incr_reset(pmp_incr* h) {
  if (!h) return fail(PMP_E_INVALID_ARG, "handle is NULL");
  hipError_t e = pmp::launch_incr_reset(h->st, h->stream);
  if (e != hipSuccess) return hip_fail(e, "state reset");
  h->len = 0;
  h->pending = false;
  return PMP_OK;
}

int pmp_incr_length(const pmp_incr* h, uint64_t* len) {
  if (!h || !len) return fail(PMP_E_INVALID_ARG, "NULL argument");
  *len = h->len;
  return PMP_OK;
}

int pmp_incr_destroy(pmp_incr* h) {
  if (!h) return PMP_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  hipError_t e1 = hipFree(h->z);
  hipError_t e2 = hipFree(h->st);
  delete h;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (e1 != hipSuccess) return hip_fail(e1, "hipFree");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFree");
  return PMP_OK;
}

}  // extern "C"
