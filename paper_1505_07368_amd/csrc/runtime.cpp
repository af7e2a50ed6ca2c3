// Host runtime of the compute actor and the C ABI of include/caf_gpu.h.
//
// The host side owns: the actor table (behaviour, signature, forwarding
// target, alive flag), request ids and futures, the slot pool and the
// arena sub-allocator that enforce the HBM budget (admission), the mailbox
// ring writer, the drain-kernel launcher, and one poller thread that turns
// completion records into resolved futures exactly once.
//
// Paper correspondence: spawn_cl and the OpenCL actor (Sec. 4.6), typed
// interfaces checked per message (Sec. 4.5), sync_send / then with unique
// request ids, errors and timeouts (Sec. 5), call-by-value messages
// (Sec. 4.4), the actor life cycle and max_msgs per run (Sec. 6).
//
// Concurrency: one mutex (`mu`) guards the actor table, the slot pool, the
// arena and the ring writer; a request takes it once in the common case.
// The poller never takes it: finished slots go into a ring that only the
// poller appends to, unreferenced futures onto a lock-free stack, and each
// later request returns a few of them to the slot pool, the future pool and
// the arena (all of them when it would otherwise be refused).  A contended
// mutex hand-off costs the poller a sleep and a wake-up per batch of
// completions.  Fields written by the submitting side and by the poller sit
// on separate cache lines, and the poller's view of a slot is kept apart
// from the arena blocks only the submitting side reads.
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "caf_internal.h"

namespace cafgpu {
hipError_t launch_plain(const KArgs& a, const Desc& d, uint32_t ntiles, hipStream_t s);
hipError_t launch_drain(const KArgs& a, hipStream_t s);
hipError_t drain_occupancy(bool full, uint32_t full_wgs, bool wide, int* blocks_per_cu);
const void* plain_kernel_fn(bool full);
}  // namespace cafgpu

using namespace cafgpu;

namespace {

constexpr uint64_t kGranule = 256;
constexpr uint32_t kMaxTemps = 6;
constexpr uint32_t kPollBatch = 256;

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Best-fit sub-allocator over the caller's arena, with coalescing.  Freed
// blocks first go onto per-size lists that the next request of that size
// takes in O(1) (serving workloads repeat a few sizes); they are merged
// into the coalescing tree when a request finds no block, so a request
// fails only if the coalesced arena cannot hold it.  Not synchronised:
// every call is made with the system mutex held.
class Arena {
 public:
  void init(uint64_t base, uint64_t bytes) {
    base_ = base;
    size_ = bytes / kGranule * kGranule;
    by_off_.clear();
    by_size_.clear();
    quick_.clear();
    quick_blocks_ = 0;
    insert(0, size_);
  }
  static uint64_t granules(uint64_t bytes) {
    const uint64_t need = (bytes + kGranule - 1) / kGranule * kGranule;
    return need ? need : kGranule;
  }
  bool alloc(uint64_t bytes, uint64_t* addr) {
    const uint64_t need = granules(bytes);
    auto q = quick_.find(need);
    if (q != quick_.end() && !q->second.empty()) {
      *addr = base_ + q->second.back();
      q->second.pop_back();
      --quick_blocks_;
    } else if (!tree_alloc(need, addr)) {
      if (!quick_blocks_) return false;
      flush_quick();
      if (!tree_alloc(need, addr)) return false;
    }
    in_use_ += need;
    if (in_use_ > peak_) peak_ = in_use_;
    return true;
  }
  void free(uint64_t addr, uint64_t bytes) {
    const uint64_t sz = granules(bytes);
    in_use_ -= sz;
    quick_[sz].push_back(addr - base_);
    if (++quick_blocks_ > kQuickMax) flush_quick();
  }
  uint64_t size() const { return size_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }

 private:
  static constexpr uint64_t kQuickMax = 1u << 16;
  bool tree_alloc(uint64_t need, uint64_t* addr) {
    auto it = by_size_.lower_bound({need, 0});
    if (it == by_size_.end()) return false;
    const uint64_t sz = it->first, off = it->second;
    erase(off, sz);
    if (sz > need) insert(off + need, sz - need);
    *addr = base_ + off;
    return true;
  }
  void flush_quick() {
    for (auto& kv : quick_)
      for (uint64_t off : kv.second) tree_free(off, kv.first);
    quick_.clear();
    quick_blocks_ = 0;
  }
  void tree_free(uint64_t off, uint64_t sz) {
    auto nx = by_off_.lower_bound(off);
    if (nx != by_off_.end() && nx->first == off + sz) {
      const uint64_t nsz = nx->second;
      erase(nx->first, nsz);
      sz += nsz;
    }
    auto pv = by_off_.lower_bound(off);
    if (pv != by_off_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        const uint64_t poff = pv->first, psz = pv->second;
        erase(poff, psz);
        off = poff;
        sz += psz;
      }
    }
    insert(off, sz);
  }
  void insert(uint64_t off, uint64_t sz) {
    by_off_[off] = sz;
    by_size_.emplace(sz, off);
  }
  void erase(uint64_t off, uint64_t sz) {
    by_off_.erase(off);
    by_size_.erase({sz, off});
  }
  uint64_t base_ = 0, size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> by_off_;                 // free blocks by offset
  std::set<std::pair<uint64_t, uint64_t>> by_size_;     // (size, offset): best fit, lowest offset
  std::unordered_map<uint64_t, std::vector<uint64_t>> quick_;  // size -> freed offsets
  uint64_t quick_blocks_ = 0;
};

struct Block {
  uint64_t addr = 0, bytes = 0;
};

struct ActorRec {
  int32_t behavior = -1;
  caf_spawn_args spawn{};
  bool alive = false;
  uint32_t seq = 0;  // next per-actor sequence number
};

size_t dtype_bytes(int32_t dt) {
  switch (dt) {
    case CAF_I32: return 4;
    case CAF_U16: return 2;
    case CAF_F32: return 4;
    case CAF_F64: return 8;
    case CAF_BF16: return 2;
    case CAF_U64: return 8;
    case CAF_U32: return 4;
  }
  return 0;
}

}  // namespace

struct caf_future {
  caf_gpu_system* sys = nullptr;
  uint64_t req_id = 0;
  std::atomic<int> state{0};  // 0 pending, 1 replied, 2 gave up (timeout)
  int32_t status = 0;
  caf_buf result{};
  uint8_t inline_data[kInlineBytes] = {};
  Block out;                  // arena reply buffer owned by this future
  std::atomic<int> refs{2};   // the caller's handle + the request in flight
  caf_future* next_retired = nullptr;  // link on the retired-future stack
  int64_t t_issue = 0, t_done = 0;
  DriveQ* q = nullptr;        // driver notification (optional)
  uint32_t tag = 0;
  bool pooled = false;
};

// What the poller needs of a slot (written at submit, cleared by the poller;
// one line per slot so neighbouring slots do not share it).
struct alignas(64) SlotInfo {
  uint64_t req_id = 0;
  caf_future* fut = nullptr;
};

// What only the submitting side needs of a slot (under mu): the arena blocks
// to return when the slot is reclaimed.
struct SlotTemps {
  Block temps[kMaxTemps];  // staged inputs, intermediate and unwanted replies
  uint32_t ntemps = 0;
};

// An instantiated graph of one message's plain launches (one kernel node per
// pipeline stage, in stream order) for one stage shape.
struct PlainGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node[1 + kMaxHops] = {};
};
using PlainShape = std::array<uint32_t, 2 + kMaxHops>;  // stage count, then (full << 31 | tiles)
constexpr size_t kMaxGraphs = 64;

struct caf_gpu_system {
  caf_gpu_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t dstream[2] = {nullptr, nullptr};  // drain launches alternate between these
  bool own_stream = false, own_dstream[2] = {false, false};
  // host memory shared with the device
  HostCtl* hctl = nullptr;
  Desc* hring = nullptr;
  Comp* comp = nullptr;
  // device memory
  DevCtl* dctl = nullptr;
  DevSlot* dslots = nullptr;
  SlotState* sstate = nullptr;
  uint32_t* tile2slot = nullptr;
  DevActor* dactors = nullptr;
  KArgs kargs{};
  uint32_t cap = 0;
  // The submitting threads and the poller thread each write their own group
  // of fields below; the groups, and every field both sides write, start on
  // their own 64-byte line, so a completion does not evict the submit
  // path's lines (the lock, the ring tail, the pools).
  // guarded by mu
  alignas(64) std::mutex mu;
  std::condition_variable cv_space;
  Arena arena;
  std::vector<ActorRec> actors;
  std::vector<SlotInfo> slots;
  std::vector<SlotTemps> slot_temps;
  std::vector<uint32_t> free_slots;
  std::vector<caf_future*> fut_pool;
  std::vector<caf_future*> all_futs;  // every future object, for shutdown
  uint64_t tail = 0;
  uint64_t req_seq = 1;
  bool shut = false;
  std::vector<uint32_t> pend_slots;        // retired, not yet returned (mu)
  std::vector<caf_future*> pend_futs;
  // Finished slots: the poller appends (single producer), reclaim() takes
  // them in order under mu.  Every slot is in it at most once, so a power
  // of two >= the slot count never overflows.
  std::vector<uint32_t> retired_ring;
  uint64_t retired_head = 0;  // mu
  std::atomic<uint64_t> st_requests{0}, st_sends{0}, st_launches{0}, st_rejected{0};
  // written by both sides
  alignas(64) std::atomic<uint64_t> outstanding{0};
  alignas(64) std::atomic<uint32_t> waiters{0};
  alignas(64) std::atomic<uint64_t> retired_tail{0};  // poller
  // Returned without mu: pushed by any thread, emptied whole under mu.
  alignas(64) std::atomic<caf_future*> retired_futs{nullptr};
  // drain kernel
  alignas(64) std::mutex launch_mu;
  std::atomic<uint32_t> launched_gen{0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  std::atomic<uint64_t> st_drain_launches{0};
  // poller
  alignas(64) std::thread poller;
  std::atomic<bool> stop_poller{false};
  uint64_t comp_head = 0;
  uint32_t ccap = 0;  // completion ring entries (power of two)
  std::atomic<uint64_t> st_completions{0}, st_dup{0}, st_swallowed{0};
  alignas(64) uint32_t mandel_tile_px = 1024;
  uint32_t gemm_tile = 0;
  uint32_t grid_full = 0, grid_light = 0;  // drain-kernel workgroups per variant
  std::atomic<bool> need_full{false};       // a GEMM actor exists
  std::atomic<bool> held{false};            // caf_gpu_hold: no new drain launch
  bool last_full = false;                   // variant of the latest drain launch (launch_mu)
  hipEvent_t handover = nullptr;            // light -> full launch ordering (launch_mu)
  std::map<PlainShape, PlainGraph> graphs;  // CAF_MODE_PLAIN_GRAPH, guarded by mu
  // CPU actors of the CPU+GPU split (offload.cpp)
  cafgpu::CpuPool* cpu_pool = nullptr;
  std::mutex offload_mu;
  bool plain() const { return cfg.mode == CAF_MODE_PLAIN || cfg.mode == CAF_MODE_PLAIN_GRAPH; }
};

namespace cafgpu {
CpuPool*& cpu_pool_of(caf_gpu_system* s) { return s->cpu_pool; }
std::mutex& offload_mu_of(caf_gpu_system* s) { return s->offload_mu; }
int device_of(const caf_gpu_system* s) { return s->device; }
}  // namespace cafgpu

namespace {

caf_future* new_future(caf_gpu_system* s) {  // mu held
  caf_future* f;
  if (!s->fut_pool.empty()) {
    f = s->fut_pool.back();
    s->fut_pool.pop_back();
  } else {
    f = new caf_future();
    s->all_futs.push_back(f);
  }
  f->pooled = false;
  f->sys = s;
  f->req_id = 0;
  f->state.store(0, std::memory_order_relaxed);
  f->status = 0;
  f->result = caf_buf{};
  f->out = Block{};
  f->refs.store(2, std::memory_order_relaxed);
  f->t_issue = f->t_done = 0;
  f->q = nullptr;
  f->tag = 0;
  return f;
}


void put_ref(caf_future* f) {  // mu not held
  if (f->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) {
    caf_gpu_system* s = f->sys;
    if (!s) {  // orphaned by caf_gpu_shutdown
      delete f;
      return;
    }
    caf_future* top = s->retired_futs.load(std::memory_order_relaxed);
    do {
      f->next_retired = top;
    } while (!s->retired_futs.compare_exchange_weak(top, f, std::memory_order_release,
                                                    std::memory_order_relaxed));
    if (s->waiters.load(std::memory_order_relaxed)) s->cv_space.notify_all();
  }
}

// Returns up to `budget` retired slots and as many futures, with their
// arena blocks, to the pools (mu held).  The retired slots published so far
// and the whole retired-future stack are moved to pending lists, so a push
// racing with this one simply waits for the next call; the budget spreads
// the work of a large burst of completions over the requests that follow
// instead of stalling one of them.
constexpr size_t kReclaimBudget = 16;
constexpr size_t kReclaimAll = ~size_t(0);

bool reclaim_pending(const caf_gpu_system* s) {
  return !s->pend_slots.empty() || !s->pend_futs.empty() ||
         s->retired_head != s->retired_tail.load(std::memory_order_relaxed) ||
         s->retired_futs.load(std::memory_order_relaxed);
}

void reclaim(caf_gpu_system* s, size_t budget) {
  {
    const uint64_t tl = s->retired_tail.load(std::memory_order_acquire);
    const uint64_t mask = s->retired_ring.size() - 1;
    for (; s->retired_head < tl; ++s->retired_head)
      s->pend_slots.push_back(s->retired_ring[s->retired_head & mask]);
  }
  if (s->retired_futs.load(std::memory_order_relaxed)) {
    caf_future* f = s->retired_futs.exchange(nullptr, std::memory_order_acquire);
    while (f) {
      s->pend_futs.push_back(f);
      f = f->next_retired;
    }
  }
  for (size_t n = 0; n < budget && !s->pend_slots.empty(); ++n) {
    const uint32_t slot = s->pend_slots.back();
    s->pend_slots.pop_back();
    SlotTemps& st = s->slot_temps[slot];
    for (uint32_t k = 0; k < st.ntemps; ++k) s->arena.free(st.temps[k].addr, st.temps[k].bytes);
    st.ntemps = 0;
    s->free_slots.push_back(slot);
  }
  for (size_t n = 0; n < budget && !s->pend_futs.empty(); ++n) {
    caf_future* f = s->pend_futs.back();
    s->pend_futs.pop_back();
    if (f->out.bytes) s->arena.free(f->out.addr, f->out.bytes);
    f->out = Block{};
    f->next_retired = nullptr;
    f->pooled = true;
    s->fut_pool.push_back(f);
  }
}

// True while the latest drain launch serves the mailbox (neither retiring
// nor exited).
bool drain_running(caf_gpu_system* s) {
  const uint32_t g = s->launched_gen.load(std::memory_order_acquire);
  if (g == 0) return false;
  const uint32_t p = g & 1u;
  return __atomic_load_n(&s->hctl->retiring[p], __ATOMIC_ACQUIRE) != g &&
         __atomic_load_n(&s->hctl->exited[p], __ATOMIC_ACQUIRE) != g;
}

// Launches the drain kernel if it is not running (ring modes).
void ensure_drain(caf_gpu_system* s, bool only_if_pending) {
  if (s->held.load(std::memory_order_acquire)) return;
  if (drain_running(s)) return;  // fast path, no lock
  std::lock_guard<std::mutex> g(s->launch_mu);
  // again under the lock: caf_gpu_hold sets the flag under it, so a caller
  // that passed the check above before a hold, and finds work pending only
  // because the held messages arrived meanwhile, launches nothing
  if (s->held.load(std::memory_order_acquire)) return;
  if (drain_running(s)) return;
  if (only_if_pending &&
      __atomic_load_n(&s->hctl->drained, __ATOMIC_ACQUIRE) >=
          __atomic_load_n(&s->hctl->tail, __ATOMIC_ACQUIRE))
    return;
  KArgs a = s->kargs;
  a.gen = s->launched_gen.load() + 1;
  a.full = s->need_full.load() ? 1u : 0u;
  a.grid = a.full ? s->grid_full : s->grid_light;
  // Launch windows are timed with events until the pool is full.
  if (s->ev_used == s->ev_pool.size() && s->ev_pool.size() < 16384) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    s->ev_pool.emplace_back(e0, e1);
  }
  // The previous launch may still be finishing its last tiles on the other
  // stream; launches cooperate through the shared counters.
  hipStream_t st = s->dstream[a.gen & 1u];
  // A light launch cannot run GEMM tiles, and its workgroups may still
  // reserve tile indices until they notice that their launch retires.  The
  // first full launch after light ones therefore starts only once every
  // earlier launch has exited: it waits for the other drain stream (and its
  // own stream orders it after the launch before that), so no light
  // workgroup is resident when a product's tiles are published.
  if (a.full && !s->last_full && a.gen > 1) {
    hipEventRecord(s->handover, s->dstream[(a.gen + 1) & 1u]);
    hipStreamWaitEvent(st, s->handover, 0);
  }
  const bool timed = s->ev_used < s->ev_pool.size();
  if (timed) hipEventRecord(s->ev_pool[s->ev_used].first, st);
  const hipError_t e = launch_drain(a, st);
  if (e != hipSuccess) {
    std::fprintf(stderr, "cafgpu: drain launch failed: %s\n", hipGetErrorString(e));
    return;
  }
  if (timed) hipEventRecord(s->ev_pool[s->ev_used++].second, st);
  s->last_full = a.full != 0;
  s->launched_gen.store(a.gen, std::memory_order_release);
  s->st_drain_launches++;
}

// Resolves a batch of completion records (poller thread).
void resolve_batch(caf_gpu_system* s, const Comp* recs, uint32_t n) {
  caf_future* futs[kPollBatch];
  const Comp* frec[kPollBatch];
  uint32_t nf = 0, valid = 0;
  uint64_t rt = s->retired_tail.load(std::memory_order_relaxed);  // this thread's own
  const uint64_t rmask = s->retired_ring.size() - 1;
  // A slot's record was written under mu before its ring entry was
  // published, and stays the poller's from its completion until reclaim()
  // hands the slot out again; clearing req_id makes a repeated record for it
  // a duplicate.
  for (uint32_t i = 0; i < n; ++i) {
    const Comp& c = recs[i];
    const uint32_t slot = (uint32_t)(c.req_id & (kMaxSlots - 1));
    if (slot >= s->cap || s->slots[slot].req_id != c.req_id) {
      s->st_dup++;
      continue;
    }
    SlotInfo& si = s->slots[slot];
    if (si.fut) {
      futs[nf] = si.fut;
      frec[nf] = &c;
      ++nf;
    }
    si.fut = nullptr;
    si.req_id = 0;
    s->retired_ring[rt++ & rmask] = slot;
    ++valid;
  }
  // the slots go back after their records are consumed (release: reclaim
  // sees the cleared fields)
  s->retired_tail.store(rt, std::memory_order_release);
  s->st_completions += valid;
  const int64_t t = now_ns();
  for (uint32_t i = 0; i < nf; ++i) {
    caf_future* f = futs[i];
    f->status = frec[i]->status;
    if (f->result.on_device == 0 && f->result.data == f->inline_data)
      std::memcpy(f->inline_data, frec[i]->data, kInlineBytes);
    f->t_done = t;
    int expect = 0;
    if (f->state.compare_exchange_strong(expect, 1, std::memory_order_acq_rel)) {
      if (f->q) {
        DriveQ* q = f->q;
        const uint64_t tl = __atomic_load_n(&q->tail, __ATOMIC_RELAXED);
        q->buf[tl & q->mask] = f->tag;
        __atomic_store_n(&q->tail, tl + 1, __ATOMIC_RELEASE);
      }
    } else {
      s->st_swallowed++;
    }
    put_ref(f);
  }
  s->outstanding.fetch_sub(valid, std::memory_order_acq_rel);
  if (s->waiters.load(std::memory_order_relaxed)) s->cv_space.notify_all();
}

void poller_main(caf_gpu_system* s) {
  hipSetDevice(s->device);
  uint32_t idle = 0;
  const uint32_t ccap = s->ccap;
  Comp batch[kPollBatch];
  while (!s->stop_poller.load(std::memory_order_relaxed)) {
    uint32_t n = 0;
    while (n < kPollBatch) {
      const Comp* c = &s->comp[s->comp_head & (ccap - 1)];
      const uint32_t lap = (uint32_t)(s->comp_head / ccap) + 1;
      if (__atomic_load_n(&c->lap, __ATOMIC_ACQUIRE) != lap) break;
      std::memcpy(&batch[n], c, sizeof(Comp));
      s->comp_head++;
      ++n;
    }
    if (n) {
      resolve_batch(s, batch, n);
      idle = 0;
      continue;
    }
    if (!s->plain() && (idle & 63) == 0) ensure_drain(s, true);
    ++idle;
    if (idle < 20000 || s->outstanding.load(std::memory_order_relaxed) != 0) {
      _mm_pause();
    } else {
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  }
}

// Reply element type / count of a behaviour, and signature checks.
struct Shape {
  int32_t dtype = CAF_F32;
  uint64_t numel = 0;
  uint32_t rows = 0, cols = 0;  // shape handed to a forwarded stage
};

int check_stage_input(const ActorRec& a, uint32_t rows, uint32_t cols, Shape* out) {
  if (a.behavior == CAF_BHV_TANH) {
    if (a.spawn.n && (a.spawn.n != rows || a.spawn.n != cols)) return CAF_E_INVALID;
    *out = Shape{CAF_F32, (uint64_t)rows * cols, rows, cols};
    return CAF_OK;
  }
  if (a.behavior == CAF_BHV_ROWSUM) {
    if (a.spawn.n && (a.spawn.n != rows || a.spawn.n != cols)) return CAF_E_INVALID;
    *out = Shape{CAF_F32, rows, rows, 1};
    return CAF_OK;
  }
  return CAF_E_INVALID;  // only f32 matrix stages can be forwarded to
}

int check_signature(const ActorRec& a, const void* args, uint64_t args_bytes, const caf_buf* in,
                    uint32_t n_in, Shape* out) {
  switch (a.behavior) {
    case CAF_BHV_NOOP:
      if (n_in != 1 || !in || in[0].dtype != CAF_I32 || in[0].numel == 0 || !in[0].data)
        return CAF_E_INVALID;
      if (in[0].numel > (1u << 30)) return CAF_E_INVALID;
      *out = Shape{CAF_I32, in[0].numel, 0, 0};
      return CAF_OK;
    case CAF_BHV_MANDELBROT: {
      if (n_in != 0 || args_bytes != sizeof(caf_mandel_args) || !args) return CAF_E_INVALID;
      const caf_mandel_args* m = (const caf_mandel_args*)args;
      if (m->max_iter < 1 || m->max_iter > 65535 || m->width == 0) return CAF_E_INVALID;
      if (m->fp != CAF_F32 && m->fp != CAF_F64) return CAF_E_INVALID;
      if ((uint64_t)m->row0 + m->rows > m->height) return CAF_E_INVALID;
      if (m->width > (1u << 20) || m->rows > (1u << 20)) return CAF_E_INVALID;
      // at most 2^32 pixels (an 8 GiB reply), so block and tile counts fit 32 bits
      if ((uint64_t)m->rows * m->width > (1ull << 32)) return CAF_E_INVALID;
      *out = Shape{a.spawn.palette_len ? CAF_U32 : CAF_U16, (uint64_t)m->rows * m->width, m->rows,
                   m->width};
      return CAF_OK;
    }
    case CAF_BHV_GEMM: {
      if (args_bytes != sizeof(caf_gemm_args) || !args || n_in != 2 || !in) return CAF_E_INVALID;
      const caf_gemm_args* g = (const caf_gemm_args*)args;
      if (g->n == 0 || g->n > 16384) return CAF_E_INVALID;
      if (g->in_dtype != CAF_F32 && g->in_dtype != CAF_BF16) return CAF_E_INVALID;
      if (a.spawn.n && a.spawn.n != g->n) return CAF_E_INVALID;
      const uint64_t nn = (uint64_t)g->n * g->n;
      for (int i = 0; i < 2; ++i)
        if (in[i].dtype != g->in_dtype || in[i].numel != nn || !in[i].data) return CAF_E_INVALID;
      *out = Shape{CAF_F32, nn, g->n, g->n};
      return CAF_OK;
    }
    case CAF_BHV_TANH:
    case CAF_BHV_ROWSUM: {
      if (args_bytes != sizeof(caf_shape_args) || !args || n_in != 1 || !in) return CAF_E_INVALID;
      const caf_shape_args* sh = (const caf_shape_args*)args;
      if (sh->rows == 0 || sh->cols == 0) return CAF_E_INVALID;
      if (in[0].dtype != CAF_F32 || !in[0].data) return CAF_E_INVALID;
      if (in[0].numel != (uint64_t)sh->rows * sh->cols) return CAF_E_INVALID;
      return check_stage_input(a, sh->rows, sh->cols, out);
    }
    case CAF_BHV_HASHCHAIN:
      if (n_in != 0 || args_bytes != sizeof(caf_hash_args) || !args) return CAF_E_INVALID;
      *out = Shape{CAF_U64, 1, 0, 0};
      return CAF_OK;
    case CAF_BHV_FAULT:
      *out = Shape{CAF_I32, 0, 0, 0};
      return CAF_OK;
  }
  return CAF_E_INVALID;
}

// Tile choice of a product (tcfg).  A system that runs the wide drain
// variant gives 256 (128 x 256 bf16 tiles) to every product that qualifies
// -- bf16 inputs, n % 32 == 0, 16-byte aligned device inputs (host inputs
// are staged into the arena, which is) -- whatever its size class asks for:
// in that variant the square tiles are calls.  Other products get their
// class's edge, 128 where that is 256.
uint32_t gemm_tile_for(const caf_gpu_system* s, const caf_gemm_args* g, const caf_buf* in) {
  const uint32_t n = g->n;
  if (s->kargs.wide && g->in_dtype == CAF_BF16 && n % 32 == 0) {
    bool aligned = true;
    for (int i = 0; i < 2; ++i)
      if (in[i].on_device && ((uintptr_t)in[i].data & 15u) != 0) aligned = false;
    if (aligned) return 256;
  }
  uint32_t t = s->gemm_tile;
  if (t == 0) {
    const uint32_t cls = n <= 64 ? 0u : n <= 128 ? 1u : n <= 256 ? 2u : 3u;
    t = s->cfg.gemm_tile_class[cls];
    if (t == 0) t = n <= 128 ? 64u : 128u;
  }
  return t == 256 ? 128u : t;
}

// Builds the descriptor of the first stage (all fields except slot, seq and
// request id).
void fill_desc(const caf_gpu_system* s, const ActorRec& a, uint32_t aidx, const void* args,
               const caf_buf* in, bool inline_in, bool inline_out, bool is_request, Desc* d) {
  std::memset(d, 0, sizeof *d);
  d->actor = aidx;
  d->behavior = (uint16_t)a.behavior;
  switch (a.behavior) {
    case CAF_BHV_MANDELBROT: {
      const caf_mandel_args* m = (const caf_mandel_args*)args;
      if (m->fp == CAF_F64) {
        d->flags |= DF_FP64;
        d->p.m64.re_min = m->re_min;
        d->p.m64.im_min = m->im_min;
        d->p.m64.step_re = m->step_re;
        d->p.m64.step_im = m->step_im;
      } else {
        // float messages: the viewport doubles are rounded to float once
        d->p.m32.re_min = (float)m->re_min;
        d->p.m32.im_min = (float)m->im_min;
        d->p.m32.step_re = (float)m->step_re;
        d->p.m32.step_im = (float)m->step_im;
      }
      d->p.m64.width = m->width;
      d->p.m64.row0 = m->row0;
      d->p.m64.rows = m->rows;
      d->p.m64.max_iter = m->max_iter;
      d->tcfg = s->mandel_tile_px;
      if (a.spawn.palette_len) {
        d->flags |= DF_RGBA;
        d->in0 = (uint64_t)(uintptr_t)a.spawn.palette;
        d->numel = a.spawn.palette_len;
      }
      break;
    }
    case CAF_BHV_GEMM: {
      const caf_gemm_args* g = (const caf_gemm_args*)args;
      if (g->in_dtype == CAF_BF16) d->flags |= DF_BF16;
      d->p.g.n = g->n;
      d->tcfg = gemm_tile_for(s, g, in);
      // bf16 products in units of four tiles, 128 x 256 ones too (half of an
      // n = 512 product; with drained products in mailbox order four ran a
      // batch 1.5-3% faster than two and 7% faster than eight, whose units
      // are too coarse to end a batch evenly); fp32 in single tiles
      d->p.g.unit = g->in_dtype != CAF_BF16 ? 1u : kGemmUnitBf16;
      break;
    }
    case CAF_BHV_TANH:
    case CAF_BHV_ROWSUM: {
      const caf_shape_args* x = (const caf_shape_args*)args;
      d->p.s.rows = x->rows;
      d->p.s.cols = x->cols;
      break;
    }
    case CAF_BHV_HASHCHAIN:
      d->p.h.x = ((const caf_hash_args*)args)->x;
      break;
    case CAF_BHV_NOOP:
      d->numel = (uint32_t)in[0].numel;
      if (inline_in) {
        d->flags |= DF_INLINE_IN;
        std::memcpy(d->p.raw, in[0].data, in[0].numel * 4);
      }
      break;
    default:
      break;
  }
  if (inline_out) d->flags |= DF_INLINE_OUT;
  if (!is_request) d->flags |= DF_SEND;
}

// Replays the graph of this stage shape with the message's arguments (mu
// held).  Returns false, launching nothing, if the shape has no graph and
// the cache is full; *err receives the HIP status otherwise.
bool launch_graph(caf_gpu_system* s, const Desc* sd, const uint32_t* nt, uint32_t nstages,
                  hipError_t* err) {
  PlainShape key{};
  key[0] = nstages;
  for (uint32_t k = 0; k < nstages; ++k)
    key[1 + k] = ((sd[k].behavior == CAF_BHV_GEMM ? 1u : 0u) << 31) | nt[k];
  auto it = s->graphs.find(key);
  hipKernelNodeParams p[1 + kMaxHops];
  void* argv[1 + kMaxHops][3];
  KArgs ka = s->kargs;
  Desc d[1 + kMaxHops];
  uint32_t n[1 + kMaxHops];
  for (uint32_t k = 0; k < nstages; ++k) {
    d[k] = sd[k];
    n[k] = nt[k];
    argv[k][0] = &ka;
    argv[k][1] = &d[k];
    argv[k][2] = &n[k];
    p[k] = hipKernelNodeParams{};
    p[k].func = const_cast<void*>(plain_kernel_fn(sd[k].behavior == CAF_BHV_GEMM));
    p[k].gridDim = dim3(nt[k]);
    p[k].blockDim = dim3(kThreads);
    p[k].sharedMemBytes = 0;
    p[k].kernelParams = argv[k];
    p[k].extra = nullptr;
  }
  hipError_t e = hipSuccess;
  if (it == s->graphs.end()) {
    if (s->graphs.size() >= kMaxGraphs) return false;
    PlainGraph g;
    e = hipGraphCreate(&g.graph, 0);
    for (uint32_t k = 0; k < nstages && e == hipSuccess; ++k)
      e = hipGraphAddKernelNode(&g.node[k], g.graph, k ? &g.node[k - 1] : nullptr, k ? 1 : 0,
                                &p[k]);
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (g.graph) hipGraphDestroy(g.graph);
      *err = e;
      return true;
    }
    it = s->graphs.emplace(key, g).first;
  } else {
    for (uint32_t k = 0; k < nstages && e == hipSuccess; ++k)
      e = hipGraphExecKernelNodeSetParams(it->second.exec, it->second.node[k], &p[k]);
  }
  if (e == hipSuccess) e = hipGraphLaunch(it->second.exec, s->stream);
  *err = e;
  return true;
}

int submit(caf_gpu_system* s, caf_actor dst, uint32_t sender, const void* args,
           uint64_t args_bytes, const caf_buf* in, uint32_t n_in, const caf_buf* out_buf,
           caf_actor forward_to, caf_future** fut, bool is_request, DriveQ* q, uint32_t tag,
           bool try_only = false) {
  (void)sender;  // FIFO per (sender, actor) follows from the single ring order
  if (!s) return CAF_E_INVALID;
  if (n_in > 2 || (n_in && !in)) return CAF_E_INVALID;
  const bool user_out = out_buf && out_buf->data;
  std::unique_lock<std::mutex> g(s->mu);
  if (s->shut) return CAF_E_INVALID;
  // ---- signature and forwarding chain (Sec. 4.5 / 4.6) ------------------
  if (dst == 0 || dst > s->actors.size()) return CAF_E_NO_ACTOR;
  const uint32_t aidx = (uint32_t)(dst - 1);
  const ActorRec a = s->actors[aidx];
  if (!a.alive) return CAF_E_NO_ACTOR;
  Shape sh, hsh[kMaxHops];
  int st = check_signature(a, args, args_bytes, in, n_in, &sh);
  if (st != CAF_OK) return st;
  uint32_t nhops = 0, hidx[kMaxHops] = {0, 0};
  int32_t hbeh[kMaxHops] = {0, 0};
  {
    caf_actor next = forward_to ? forward_to : a.spawn.forward_to;
    Shape prev = sh;
    while (next) {
      if (nhops == kMaxHops) return CAF_E_INVALID;
      if (next > s->actors.size()) return CAF_E_NO_ACTOR;
      const ActorRec& h = s->actors[next - 1];
      if (!h.alive) return CAF_E_NO_ACTOR;
      if (prev.dtype != CAF_F32 || prev.rows == 0) return CAF_E_INVALID;
      st = check_stage_input(h, prev.rows, prev.cols, &hsh[nhops]);
      if (st != CAF_OK) return st;
      hidx[nhops] = (uint32_t)(next - 1);
      hbeh[nhops] = h.behavior;
      prev = hsh[nhops];
      ++nhops;
      next = h.spawn.forward_to;
    }
  }
  const Shape& final_shape = nhops ? hsh[nhops - 1] : sh;
  const uint64_t final_bytes = final_shape.numel * dtype_bytes(final_shape.dtype);
  const bool inline_in =
      a.behavior == CAF_BHV_NOOP && !in[0].on_device && in[0].numel * 4 <= kInlineBytes;
  const bool inline_out = nhops == 0 &&
                          (a.behavior == CAF_BHV_NOOP || a.behavior == CAF_BHV_HASHCHAIN) &&
                          final_bytes <= kInlineBytes && !user_out;
  if (user_out && (!out_buf->on_device || out_buf->dtype != final_shape.dtype ||
                   out_buf->numel != final_shape.numel))
    return CAF_E_INVALID;
  Desc d;
  fill_desc(s, a, aidx, args, in, inline_in, inline_out, is_request, &d);
  if (desc_ntiles(d) > kTileMapCap / 4) return CAF_E_INVALID;
  for (uint32_t h = 0; h < nhops; ++h)
    d.hop_actor[h] = ((uint32_t)hbeh[h] << 16) | (hidx[h] + 1);

  // ---- admission: a slot plus every arena buffer the message needs ------
  // A message whose buffers together exceed the whole arena can never be
  // admitted: refused at once, also in blocking mode (waiting would never end).
  {
    uint64_t need = 0;
    for (uint32_t i = 0; i < n_in; ++i)
      if (!in[i].on_device && !(inline_in && i == 0))
        need += Arena::granules(in[i].numel * dtype_bytes(in[i].dtype));
    for (uint32_t k = 0; k <= nhops; ++k) {
      const Shape& shk = k == 0 ? sh : hsh[k - 1];
      if (k == nhops && (inline_out || user_out)) continue;
      const uint64_t bytes = shk.numel * dtype_bytes(shk.dtype);
      need += Arena::granules(bytes ? bytes : 4);
    }
    if (need > s->arena.size()) {
      s->st_rejected++;
      return CAF_E_OVERLOAD;
    }
  }
  Block staged[2];
  Block sout[1 + kMaxHops];
  uint32_t slot = 0;
  bool reclaim_all = false;
  for (;;) {
    reclaim(s, reclaim_all ? kReclaimAll : kReclaimBudget);
    bool ok = !s->free_slots.empty();
    auto take = [&](uint64_t bytes, Block* b) {
      if (!ok) return;
      uint64_t addr;
      if (!s->arena.alloc(bytes, &addr)) {
        ok = false;
        return;
      }
      *b = Block{addr, bytes};
    };
    for (uint32_t i = 0; i < n_in; ++i)
      if (!in[i].on_device && !(inline_in && i == 0))
        take(in[i].numel * dtype_bytes(in[i].dtype), &staged[i]);
    for (uint32_t k = 0; k <= nhops; ++k) {
      const Shape& shk = k == 0 ? sh : hsh[k - 1];
      if (k == nhops && (inline_out || user_out)) continue;
      const uint64_t bytes = shk.numel * dtype_bytes(shk.dtype);
      take(bytes ? bytes : 4, &sout[k]);
    }
    if (ok) {
      slot = s->free_slots.back();
      s->free_slots.pop_back();
      break;
    }
    for (auto& b : staged)
      if (b.bytes) s->arena.free(b.addr, b.bytes), b = Block{};
    for (auto& b : sout)
      if (b.bytes) s->arena.free(b.addr, b.bytes), b = Block{};
    if (!reclaim_all && reclaim_pending(s)) {
      reclaim_all = true;  // everything finished goes back before refusing
      continue;
    }
    if (try_only) return kTryLater;  // the caller waits and retries: not a refusal
    if (!s->cfg.blocking) {
      s->st_rejected++;
      return CAF_E_OVERLOAD;
    }
    s->waiters.fetch_add(1);
    s->cv_space.wait_for(g, std::chrono::milliseconds(1));
    s->waiters.fetch_sub(1);
    if (s->shut) return CAF_E_QUIT;
  }
  uint64_t stage_out[1 + kMaxHops] = {0, 0, 0};
  for (uint32_t k = 0; k <= nhops; ++k) stage_out[k] = sout[k].addr;
  if (user_out) stage_out[nhops] = (uint64_t)(uintptr_t)out_buf->data;

  // ---- inputs: device pointers as given; host inputs are copied before
  // the message becomes visible to the device (call-by-value, Sec. 4.4)
  uint64_t inptr[2] = {0, 0};
  bool staging = false;
  for (uint32_t i = 0; i < n_in; ++i) {
    if (inline_in && i == 0) continue;
    if (in[i].on_device) inptr[i] = (uint64_t)(uintptr_t)in[i].data;
    else {
      inptr[i] = staged[i].addr;
      staging = true;
    }
  }
  auto release_all = [&]() {
    for (auto& b : staged)
      if (b.bytes) s->arena.free(b.addr, b.bytes);
    for (auto& b : sout)
      if (b.bytes) s->arena.free(b.addr, b.bytes);
    s->free_slots.push_back(slot);
  };
  if (staging) {
    g.unlock();
    bool ok = true;
    for (uint32_t i = 0; i < n_in; ++i)
      if (staged[i].bytes &&
          hipMemcpy((void*)(uintptr_t)staged[i].addr, in[i].data, staged[i].bytes,
                    hipMemcpyHostToDevice) != hipSuccess)
        ok = false;
    g.lock();
    if (!ok) {
      release_all();
      return CAF_E_DEVICE;
    }
    if (!s->actors[aidx].alive || s->shut) {
      release_all();
      return CAF_E_NO_ACTOR;
    }
  }
  if (n_in) d.in0 = inptr[0];  // else fill_desc's (a colour palette, or 0)
  d.in1 = inptr[1];
  d.out = stage_out[0];
  for (uint32_t h = 0; h < nhops; ++h) d.hop_out[h] = stage_out[h + 1];

  // ---- register the request and enqueue it in call order ---------------
  caf_future* f = nullptr;
  if (is_request) {
    f = new_future(s);
    f->result.dtype = final_shape.dtype;
    f->result.numel = final_shape.numel;
    if (inline_out) {
      f->result.data = f->inline_data;
      f->result.on_device = 0;
    } else {
      f->result.data = (void*)(uintptr_t)stage_out[nhops];
      f->result.on_device = 1;
    }
    if (!user_out) f->out = sout[nhops];
    f->q = q;
    f->tag = tag;
  }
  const uint64_t rid = (s->req_seq++ << kSlotBits) | slot;
  d.req_id = rid;
  d.slot = slot;
  // Only stateful messages take a number: the device applies them to the
  // actor's state strictly in this order (other behaviours never wait on it).
  if (a.behavior == CAF_BHV_HASHCHAIN) d.seq = s->actors[aidx].seq++;
  SlotInfo& si = s->slots[slot];
  si.req_id = rid;
  si.fut = f;
  SlotTemps& stt = s->slot_temps[slot];
  stt.ntemps = 0;
  for (auto& b : staged)
    if (b.bytes) stt.temps[stt.ntemps++] = b;
  for (uint32_t k = 0; k <= nhops; ++k)
    if (sout[k].bytes && !(f && k == nhops)) stt.temps[stt.ntemps++] = sout[k];
  if (f) {
    f->req_id = rid;
    f->t_issue = now_ns();
  }
  s->outstanding.fetch_add(1, std::memory_order_acq_rel);
  if (is_request) s->st_requests++;
  else s->st_sends++;
  if (s->plain()) {
    // One launch per stage; the stages of a pipeline follow in stream order.
    Desc sdesc[1 + kMaxHops];
    uint32_t snt[1 + kMaxHops];
    for (uint32_t k = 0; k <= nhops; ++k) {
      Desc sd = d;
      if (k > 0) {
        const Shape& ps = k == 1 ? sh : hsh[k - 2];
        sd.actor = hidx[k - 1];
        sd.behavior = (uint16_t)hbeh[k - 1];
        sd.in0 = stage_out[k - 1];
        sd.in1 = 0;
        sd.out = stage_out[k];
        std::memset(sd.p.raw, 0, sizeof sd.p.raw);
        sd.p.s.rows = ps.rows;
        sd.p.s.cols = ps.cols;
        sd.flags = (uint16_t)(d.flags & DF_SEND);
        sd.tcfg = 0;
        sd.seq = 0;  // pipeline stages keep no state
      }
      sd.hop_actor[0] = sd.hop_actor[1] = 0;
      if (k < nhops) sd.flags |= DF_NO_COMPLETE;
      sdesc[k] = sd;
      snt[k] = desc_ntiles(sd);
    }
    hipError_t e = hipSuccess;
    if (s->cfg.mode != CAF_MODE_PLAIN_GRAPH || !launch_graph(s, sdesc, snt, nhops + 1, &e)) {
      for (uint32_t k = 0; k <= nhops && e == hipSuccess; ++k)
        e = launch_plain(s->kargs, sdesc[k], snt[k], s->stream);
    }
    s->st_launches += nhops + 1;
    if (e != hipSuccess) std::fprintf(stderr, "cafgpu: launch failed: %s\n", hipGetErrorString(e));
  } else {
    std::memcpy(&s->hring[s->tail % s->cap], &d, sizeof d);
    s->tail += 1;
    __atomic_store_n(&s->hctl->tail, s->tail, __ATOMIC_RELEASE);
  }
  g.unlock();
  if (!s->plain()) ensure_drain(s, false);
  if (fut) *fut = f;
  return CAF_OK;
}

}  // namespace

int cafgpu_request_tagged(caf_gpu_system* s, caf_actor dst, uint32_t sender, const void* args,
                          uint64_t args_bytes, const caf_buf* in, uint32_t n_in,
                          const caf_buf* out_or_null, caf_actor forward_to, caf_future** fut,
                          DriveQ* q, uint32_t tag, bool try_only) {
  if (!fut) return CAF_E_INVALID;
  *fut = nullptr;
  try {
    return submit(s, dst, sender, args, args_bytes, in, n_in, out_or_null, forward_to, fut,
                  true, q, tag, try_only);
  } catch (...) {  // thrown before the message is published: nothing is pending
    return CAF_E_OVERLOAD;
  }
}

int64_t cafgpu_future_issue_ns(const caf_future* f) { return f->t_issue; }
bool cafgpu_blocking(const caf_gpu_system* s) { return s->cfg.blocking != 0; }
int64_t cafgpu_future_done_ns(const caf_future* f) { return f->t_done; }

extern "C" {

const char* caf_gpu_strerror(int st) {
  switch (st) {
    case CAF_OK: return "ok";
    case CAF_E_INVALID: return "invalid argument or signature mismatch";
    case CAF_E_NO_ACTOR: return "no such actor (or it quit)";
    case CAF_E_OVERLOAD: return "admission refused: HBM budget or mailbox full";
    case CAF_E_TIMEOUT: return "timed out";
    case CAF_E_DEVICE: return "device error";
    case CAF_E_QUIT: return "actor quit before handling the message";
    case CAF_E_FAULT: return "handler reported failure";
  }
  return "unknown status";
}

int caf_gpu_init(const caf_gpu_config* cfg, caf_gpu_system** out) {
  if (!cfg || !out || !cfg->arena || cfg->arena_bytes < (1u << 16)) return CAF_E_INVALID;
  if (cfg->mode < CAF_MODE_PLAIN || cfg->mode > CAF_MODE_PLAIN_GRAPH) return CAF_E_INVALID;
  const uint32_t cap = cfg->ring_slots ? cfg->ring_slots : 4096;
  const uint32_t mb = cfg->max_batch ? cfg->max_batch : 1024;
  if (cap < 2 || cap > kMaxSlots || mb > kMaxBatch) return CAF_E_INVALID;
  // Plain launches carry one message each, so their tiles are smaller to
  // give one launch enough workgroups.
  const uint32_t mpx = cfg->mandel_tile_px ? cfg->mandel_tile_px
                                           : (cfg->mode == CAF_MODE_PLAIN ||
                                                      cfg->mode == CAF_MODE_PLAIN_GRAPH
                                                  ? 512u
                                                  : 1024u);
  if (mpx % 256 != 0 || mpx > 65536) return CAF_E_INVALID;
  auto tile_ok = [](uint32_t t) { return t == 0 || t == 64 || t == 128 || t == 256; };
  if (!tile_ok(cfg->gemm_tile)) return CAF_E_INVALID;
  for (uint32_t t : cfg->gemm_tile_class)
    if (!tile_ok(t)) return CAF_E_INVALID;
  if (cfg->grouping != CAF_GROUP_FIFO && cfg->grouping != CAF_GROUP_LPT &&
      cfg->grouping != CAF_GROUP_KIND)
    return CAF_E_INVALID;
  if (cfg->full_wgs_per_cu != 0 && cfg->full_wgs_per_cu != 2 && cfg->full_wgs_per_cu != 3)
    return CAF_E_INVALID;
  if (hipSetDevice(cfg->device) != hipSuccess) return CAF_E_DEVICE;
  // once per device: the address of this device's no-alloc staging array
  if (const int st = cafgpu::offload_stage_setup(cfg->device); st != CAF_OK) return st;
  caf_gpu_system* s = new caf_gpu_system();
  s->cfg = *cfg;
  s->device = cfg->device;
  s->cap = cap;
  s->mandel_tile_px = mpx;
  s->gemm_tile = cfg->gemm_tile;
  s->kargs.full_wgs = cfg->full_wgs_per_cu == 3 ? 3u : 2u;
  {
    // 128 x 256 bf16 tiles: asked for by a tile choice of 256, in a ring
    // mode with two full workgroups per CU (their LDS holds the tile's
    // three stages); full launches then use the wide variant.
    bool asked = cfg->gemm_tile == 256;
    for (uint32_t t : cfg->gemm_tile_class) asked = asked || t == 256;
    const bool ring = cfg->mode != CAF_MODE_PLAIN && cfg->mode != CAF_MODE_PLAIN_GRAPH;
    s->kargs.wide = asked && ring && s->kargs.full_wgs == 2 ? 1u : 0u;
  }
  s->arena.init((uint64_t)(uintptr_t)cfg->arena, cfg->arena_bytes);
  bool ok = true;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess) {
      std::fprintf(stderr, "cafgpu: init: %s\n", hipGetErrorString(e));
      ok = false;
    }
  };
  if (cfg->stream) s->stream = (hipStream_t)cfg->stream;
  else {
    chk(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->own_stream = true;
  }
  if (cfg->drain_stream) s->dstream[0] = (hipStream_t)cfg->drain_stream;
  else {
    chk(hipStreamCreateWithFlags(&s->dstream[0], hipStreamNonBlocking));
    s->own_dstream[0] = true;
  }
  chk(hipStreamCreateWithFlags(&s->dstream[1], hipStreamNonBlocking));
  s->own_dstream[1] = true;
  chk(hipEventCreateWithFlags(&s->handover, hipEventDisableTiming));
  const unsigned hflags = hipHostMallocCoherent | hipHostMallocMapped;
  chk(hipHostMalloc((void**)&s->hctl, sizeof(HostCtl), hflags));
  chk(hipHostMalloc((void**)&s->hring, sizeof(Desc) * cap, hflags));
  // Completion ring: a power of two >= the slot count (at most one
  // unconsumed record per slot), so the device indexes it with a mask.
  s->ccap = 1;
  while (s->ccap < cap) s->ccap <<= 1;
  chk(hipHostMalloc((void**)&s->comp, sizeof(Comp) * s->ccap, hflags));
  chk(hipMalloc((void**)&s->dctl, sizeof(DevCtl)));
  chk(hipMalloc((void**)&s->dslots, sizeof(DevSlot) * cap));
  chk(hipMalloc((void**)&s->sstate, sizeof(SlotState) * cap));
  chk(hipMalloc((void**)&s->tile2slot, sizeof(uint32_t) * kTileMapCap));
  chk(hipMalloc((void**)&s->dactors, sizeof(DevActor) * kMaxActors));
  if (ok) {
    std::memset(s->hctl, 0, sizeof(HostCtl));
    std::memset(s->hring, 0, sizeof(Desc) * cap);
    std::memset(s->comp, 0, sizeof(Comp) * s->ccap);
    chk(hipMemset(s->dctl, 0, sizeof(DevCtl)));
    chk(hipMemset(s->dslots, 0, sizeof(DevSlot) * cap));
    chk(hipMemset(s->sstate, 0, sizeof(SlotState) * cap));
    chk(hipMemset(s->dactors, 0, sizeof(DevActor) * kMaxActors));
    chk(hipDeviceSynchronize());
  }
  int rate_khz = 100000;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, cfg->device) !=
          hipSuccess ||
      rate_khz <= 0)
    rate_khz = 100000;
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
  // Default grid: every workgroup resident (the kernel never needs that,
  // but it is the most work in flight).
  int occ_full = 1, occ_light = 1;
  if (ok) chk(drain_occupancy(true, s->kargs.full_wgs, s->kargs.wide != 0, &occ_full));
  if (ok) chk(drain_occupancy(false, s->kargs.full_wgs, false, &occ_light));
  if (occ_full < 1) occ_full = 1;
  if (occ_light < 1) occ_light = 1;
  s->grid_full = cfg->grid ? cfg->grid : (uint32_t)(cus * occ_full);
  s->grid_light = cfg->grid ? cfg->grid : (uint32_t)(cus * occ_light);
  if (!ok) {
    delete s;
    return CAF_E_DEVICE;
  }
  try {
    s->actors.reserve(kMaxActors);
    s->slots.resize(cap);
    s->slot_temps.resize(cap);
    size_t rcap = 1;
    while (rcap < cap) rcap <<= 1;
    s->retired_ring.resize(rcap);
    s->free_slots.reserve(cap);
    s->pend_slots.reserve(cap);
  } catch (...) {  // no exception crosses the C ABI
    caf_gpu_shutdown(s);
    return CAF_E_DEVICE;
  }
  for (uint32_t i = 0; i < cap; ++i) s->free_slots.push_back(cap - 1 - i);
  // Futures for the first requests, so that a request rarely allocates one
  // (caf_offload_mandel_noalloc's requests come from here).
  try {
    for (uint32_t i = 0; i < std::min(cap, 1024u); ++i) {
      caf_future* f = new caf_future();
      f->pooled = true;
      s->all_futs.push_back(f);
      s->fut_pool.push_back(f);
    }
  } catch (...) {
    caf_gpu_shutdown(s);
    return CAF_E_OVERLOAD;
  }
  KArgs& a = s->kargs;
  a.hctl = s->hctl;
  a.hring = s->hring;
  a.comp = s->comp;
  a.dctl = s->dctl;
  a.slots = s->dslots;
  a.sstate = s->sstate;
  a.tile2slot = s->tile2slot;
  a.actors = s->dactors;
  a.cap = cap;
  a.ccap = s->ccap;
  a.max_batch = mb;
  const uint64_t idle_us =
      cfg->idle_exit_us ? cfg->idle_exit_us : (cfg->mode == CAF_MODE_BATCHED ? 50 : 200000);
  a.idle_ticks = idle_us * (uint64_t)rate_khz / 1000;
  a.wait_ticks = 2000ull * (uint64_t)rate_khz;  // 2 s
  a.exit_on_empty = cfg->mode == CAF_MODE_BATCHED ? 1u : 0u;
  a.grouping = (uint32_t)cfg->grouping;
  a.grid = s->grid_full;
  a.full = 1;
  try {
    s->poller = std::thread(poller_main, s);
  } catch (...) {
    caf_gpu_shutdown(s);
    return CAF_E_DEVICE;
  }
  *out = s;
  return CAF_OK;
}

int caf_gpu_spawn(caf_gpu_system* s, int32_t behavior, const caf_spawn_args* args,
                  caf_actor* out) {
  if (!s || !out) return CAF_E_INVALID;
  if (behavior < CAF_BHV_NOOP || behavior > CAF_BHV_FAULT) return CAF_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->shut) return CAF_E_INVALID;
  if (s->actors.size() >= kMaxActors) return CAF_E_OVERLOAD;
  ActorRec a;
  a.behavior = behavior;
  if (args) a.spawn = *args;
  if (a.spawn.palette_len || a.spawn.palette) {
    if (behavior != CAF_BHV_MANDELBROT || !a.spawn.palette || a.spawn.palette_len == 0 ||
        a.spawn.palette_len > 65536)
      return CAF_E_INVALID;
  }
  if (a.spawn.forward_to &&
      (a.spawn.forward_to > s->actors.size() || !s->actors[a.spawn.forward_to - 1].alive))
    return CAF_E_INVALID;
  a.alive = true;
  if (behavior == CAF_BHV_GEMM) s->need_full.store(true);
  const uint32_t idx = (uint32_t)s->actors.size();
  s->actors.push_back(a);
  __atomic_fetch_or(&s->hctl->alive[idx >> 5], 1u << (idx & 31), __ATOMIC_SEQ_CST);
  *out = idx + 1;
  return CAF_OK;
}

int caf_gpu_become(caf_gpu_system* s, caf_actor actor, int32_t behavior,
                   const caf_spawn_args* args) {
  if (!s) return CAF_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->shut) return CAF_E_INVALID;
  if (actor == 0 || actor > s->actors.size() || !s->actors[actor - 1].alive)
    return CAF_E_NO_ACTOR;
  if (behavior < CAF_BHV_NOOP || behavior > CAF_BHV_FAULT) return CAF_E_INVALID;
  caf_spawn_args sp{};
  if (args) sp = *args;
  if ((sp.palette_len || sp.palette) &&
      (behavior != CAF_BHV_MANDELBROT || !sp.palette || sp.palette_len == 0 ||
       sp.palette_len > 65536))
    return CAF_E_INVALID;
  if (sp.forward_to && (sp.forward_to > s->actors.size() || !s->actors[sp.forward_to - 1].alive))
    return CAF_E_INVALID;
  // Every later request is checked against, and carries, the new behaviour;
  // those already submitted carry the old one.  The device state and the
  // stateful sequence continue.
  ActorRec& a = s->actors[actor - 1];
  a.behavior = behavior;
  a.spawn = sp;
  if (behavior == CAF_BHV_GEMM) s->need_full.store(true);
  return CAF_OK;
}

int caf_gpu_send(caf_gpu_system* s, caf_actor dst, uint32_t sender, const void* args,
                 uint64_t args_bytes, const caf_buf* in, uint32_t n_in) {
  try {
    return submit(s, dst, sender, args, args_bytes, in, n_in, nullptr, 0, nullptr, false,
                  nullptr, 0);
  } catch (...) {  // host memory exhausted: no exception crosses the C ABI
    return CAF_E_OVERLOAD;
  }
}

int caf_gpu_request(caf_gpu_system* s, caf_actor dst, uint32_t sender, const void* args,
                    uint64_t args_bytes, const caf_buf* in, uint32_t n_in,
                    const caf_buf* out_or_null, caf_actor forward_to, caf_future** fut) {
  if (!fut) return CAF_E_INVALID;
  *fut = nullptr;
  try {
    return submit(s, dst, sender, args, args_bytes, in, n_in, out_or_null, forward_to, fut,
                  true, nullptr, 0);
  } catch (...) {  // host memory exhausted: no exception crosses the C ABI
    return CAF_E_OVERLOAD;
  }
}

int caf_future_poll(caf_future* f, caf_buf* result, int32_t* reply_status) {
  if (!f) return CAF_E_INVALID;
  const int st = f->state.load(std::memory_order_acquire);
  if (st == 0) return 0;
  if (st == 2) {
    if (reply_status) *reply_status = CAF_E_TIMEOUT;
    if (result) *result = caf_buf{nullptr, 0, f->result.dtype, 0};
    return 1;
  }
  if (reply_status) *reply_status = f->status;
  if (result) *result = f->result;
  return 1;
}

int caf_future_wait(caf_future* f, int64_t timeout_ns, caf_buf* result, int32_t* reply_status) {
  if (!f) return CAF_E_INVALID;
  const int64_t t0 = now_ns();
  uint32_t spins = 0;
  for (;;) {
    if (caf_future_poll(f, result, reply_status) == 1)
      return f->state.load(std::memory_order_acquire) == 2 ? CAF_E_TIMEOUT : CAF_OK;
    if (timeout_ns >= 0 && now_ns() - t0 >= timeout_ns) {
      int expect = 0;
      if (f->state.compare_exchange_strong(expect, 2)) {
        if (reply_status) *reply_status = CAF_E_TIMEOUT;
        if (result) *result = caf_buf{nullptr, 0, f->result.dtype, 0};
        return CAF_E_TIMEOUT;
      }
      continue;  // resolved concurrently
    }
    if (++spins < 4096) _mm_pause();
    else std::this_thread::yield();
  }
}

uint64_t caf_future_id(const caf_future* f) { return f ? f->req_id : 0; }

void caf_future_release(caf_future* f) {
  if (f) put_ref(f);
}

int caf_gpu_quit(caf_gpu_system* s, caf_actor actor, uint32_t /*exit_reason*/) {
  if (!s) return CAF_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  if (actor == 0 || actor > s->actors.size() || !s->actors[actor - 1].alive)
    return CAF_E_NO_ACTOR;
  const uint32_t idx = (uint32_t)(actor - 1);
  s->actors[idx].alive = false;
  __atomic_fetch_and(&s->hctl->alive[idx >> 5], ~(1u << (idx & 31)), __ATOMIC_SEQ_CST);
  return CAF_OK;
}

int caf_gpu_hold(caf_gpu_system* s, int32_t hold) {
  if (!s) return CAF_E_INVALID;
  if (s->plain()) return CAF_E_INVALID;  // plain forms launch at submit time
  {
    // under the launch lock: no launch decided before the hold starts after it
    std::lock_guard<std::mutex> g(s->launch_mu);
    s->held.store(hold != 0, std::memory_order_release);
  }
  if (!hold) ensure_drain(s, true);  // one launch for everything that waited
  return CAF_OK;
}

int caf_gpu_drain(caf_gpu_system* s, int64_t timeout_ns) {
  if (!s) return CAF_E_INVALID;
  const int64_t t0 = now_ns();
  uint32_t spins = 0;
  while (s->outstanding.load() != 0) {
    if (timeout_ns >= 0 && now_ns() - t0 > timeout_ns) return CAF_E_TIMEOUT;
    if (++spins < 4096) _mm_pause();
    else std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  return CAF_OK;
}

int caf_gpu_get_stats(caf_gpu_system* s, caf_gpu_stats* o) {
  if (!s || !o) return CAF_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  reclaim(s, kReclaimAll);  // so that the arena figures count finished requests as freed
  o->requests = s->st_requests;
  o->sends = s->st_sends;
  o->completions = s->st_completions;
  o->launches = s->st_launches;
  o->drain_launches = s->st_drain_launches;
  o->duplicate_completions = s->st_dup;
  o->swallowed = s->st_swallowed;
  o->arena_in_use = s->arena.in_use();
  o->arena_peak = s->arena.peak();
  o->rejected = s->st_rejected;
  o->device_drained = __atomic_load_n(&s->hctl->drained, __ATOMIC_ACQUIRE);
  o->outstanding = s->outstanding.load();
  return CAF_OK;
}

double caf_gpu_drain_kernel_ms(caf_gpu_system* s, uint64_t* launches) {
  if (!s) return -1.0;
  std::lock_guard<std::mutex> g(s->launch_mu);
  hipStreamSynchronize(s->dstream[0]);
  hipStreamSynchronize(s->dstream[1]);
  double total = 0.0;
  for (size_t i = 0; i < s->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev_pool[i].first, s->ev_pool[i].second) == hipSuccess)
      total += ms;
  }
  if (launches) *launches = s->ev_used;
  s->ev_used = 0;
  return total;
}

int caf_gpu_shutdown(caf_gpu_system* s) {
  if (!s) return CAF_E_INVALID;
  {
    // a CPU+GPU split in progress finishes first; then its workers go
    std::lock_guard<std::mutex> g(s->offload_mu);
    cafgpu::cpu_pool_destroy(s->cpu_pool);
    s->cpu_pool = nullptr;
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->shut = true;
  }
  s->cv_space.notify_all();
  __atomic_store_n(&s->hctl->stop, 1u, __ATOMIC_SEQ_CST);
  hipStreamSynchronize(s->dstream[0]);
  hipStreamSynchronize(s->dstream[1]);
  hipStreamSynchronize(s->stream);
  // Let the poller collect what the device finished, then stop it.
  const int64_t t0 = now_ns();
  while (s->outstanding.load() != 0 && now_ns() - t0 < 200000000LL) std::this_thread::yield();
  s->stop_poller = true;
  if (s->poller.joinable()) s->poller.join();
  // Anything left never reached the device: answer it.  Futures the caller
  // still holds stay readable and are freed by caf_future_release.
  for (size_t i = 0; i < s->slots.size(); ++i) {
    SlotInfo& si = s->slots[i];
    if (!si.req_id) continue;
    if (si.fut) {
      si.fut->status = CAF_E_QUIT;
      int expect = 0;
      si.fut->state.compare_exchange_strong(expect, 1);
      si.fut->refs.fetch_sub(1);  // the request in flight is gone
    }
    si = SlotInfo();
  }
  for (caf_future* f : s->all_futs) {
    if (f->pooled || f->refs.load() <= 0) {
      delete f;
    } else {
      f->sys = nullptr;
      f->out = Block{};
    }
  }
  for (auto& e : s->ev_pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  if (s->handover) hipEventDestroy(s->handover);
  for (auto& kv : s->graphs) {
    hipGraphExecDestroy(kv.second.exec);
    hipGraphDestroy(kv.second.graph);
  }
  hipFree(s->dctl);
  hipFree(s->dslots);
  hipFree(s->sstate);
  hipFree(s->tile2slot);
  hipFree(s->dactors);
  hipHostFree(s->hctl);
  hipHostFree(s->hring);
  hipHostFree(s->comp);
  if (s->own_stream) hipStreamDestroy(s->stream);
  for (int i = 0; i < 2; ++i)
    if (s->own_dstream[i]) hipStreamDestroy(s->dstream[i]);
  delete s;
  return CAF_OK;
}

}  // extern "C"
