// Device side of the compute actor (gfx950).
//
// Two kernels share the work-tile functions of tiles.h and one completion
// protocol:
//
//  * plain_kernel -- one launch per message (the baseline form): the
//    message's descriptor travels as a kernel argument, one workgroup per
//    work tile.
//
//  * drain_kernel -- the mailbox drain.  Messages sit in a host-written
//    mailbox ring (pinned, coherent host memory).  A workgroup that finds
//    no claimable work (one of a few sentinels, or one that just finished
//    work, holds a reservation or sees a backlog: see drain_body) takes the
//    drain lock, reads the ring tail, copies up
//    to max_batch entries (the paper's max_msgs per scheduling slot, Sec. 6)
//    into device-resident slots, checks each actor is alive, groups the
//    batch (by behaviour, largest GEMMs first, or mailbox order), prefix-sums
//    the per-message work-tile counts into one global tile sequence and
//    publishes it (the drainer reserving first).  Every workgroup claims
//    tiles of that sequence with a fetch_add on a claim cursor (see
//    "claiming work tiles" below), and no workgroup ever waits for one that
//    may not be resident; consecutive claimed tiles of one GEMM (in work
//    units of whole output tiles) run as one stream of k slices, those of one
//    Mandelbrot message as one range of pixel blocks.  Stateful hash-chain entries are applied by the
//    drainer itself, in mailbox order, while it holds the lock.  The
//    workgroup finishing a message's last tile either publishes its reply
//    (a completion record in host memory, released at system scope) or
//    forwards the reply to the next actor of a pipeline on the device (no
//    host round trip): a stage of at most kInlineStageTiles tiles runs in
//    that workgroup at once, a larger one is published as new work tiles.
//
//    A launch retires as a whole once no drain pass has taken a message for
//    idle_ticks and every published tile is claimed: a sentinel's next pass
//    that finds the mailbox empty sets the retire flag under the drain lock
//    (batched mode: tens of microseconds, so one launch serves one burst;
//    persistent mode: a long idle period); or at the stop flag.  Launches alternate between
//    two streams, so a new launch can start while the previous one finishes
//    its last tiles; launches share all counters and cooperate.  Every
//    device-side wait is bounded by wait_ticks of the wall clock.
//
// Requests are FIFO per (sender, actor) because the host appends to the
// ring in call order and the drain preserves each actor's relative order.
// A stateful update (the hash chain) that runs as a tile -- one launch per
// message, or an entry the drainer could not apply in sequence -- waits for
// its predecessor's sequence number before touching device-resident state.
#pragma clang fp contract(off)

#include "caf_internal.h"
#include "tiles.h"

// Rarely executed paths are kept out of line so their registers do not add
// to the tile loop's.
#ifndef CAF_RARE
#define CAF_RARE __device__ __noinline__
#endif

namespace cafgpu {

// Kernel arguments are read in place from the kernarg segment (the constant
// address space): handing the by-value parameter to an out-of-line function
// by reference would make every lane copy it into scratch memory.  KArgs is
// the first parameter of every kernel here, so it starts the segment.
typedef __attribute__((address_space(4))) const KArgs KArgsC;
__device__ __forceinline__ KArgsC& kargs() {
  return *(KArgsC*)(__builtin_amdgcn_kernarg_segment_ptr());
}

// ---- scoped memory operations ---------------------------------------------

template <typename T>
__device__ __forceinline__ T ld_sys(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ T ld_sys_acq(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_sys_rel(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_dev_acq(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev_rel(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ bool cas_dev(T* p, T& expected, T desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

__device__ __forceinline__ void backoff_sleep(uint32_t rounds) {
  for (uint32_t i = 0; i < rounds; ++i) __builtin_amdgcn_s_sleep(32);
}

__device__ __forceinline__ bool actor_alive(const HostCtl* h, uint32_t actor) {
  return (ld_sys(&h->alive[actor >> 5]) >> (actor & 31)) & 1u;
}

// ---- completion -------------------------------------------------------------

// Publishes one reply notification to the host at completion position
// `pos` (thread-level).
__device__ void write_completion_at(KArgsC& a, uint64_t pos, uint64_t req_id, int32_t status,
                                    const uint8_t* data) {
  Comp* c = &a.comp[pos & (a.ccap - 1u)];  // ccap is a power of two
  st_sys(&c->req_id, req_id);
  st_sys(&c->status, status);
  uint32_t* dst = reinterpret_cast<uint32_t*>(c->data);
  for (int i = 0; i < 4; ++i) {
    uint32_t v = 0;
    if (data) v = reinterpret_cast<const uint32_t*>(data)[i];
    st_sys(dst + i, v);
  }
  st_sys_rel(&c->lap, (uint32_t)(pos >> __builtin_ctz(a.ccap)) + 1u);
}

// Publishes one reply notification at the next completion position.
__device__ void write_completion(KArgsC& a, uint64_t req_id, int32_t status,
                                 const uint8_t* data) {
  const uint64_t pos = __hip_atomic_fetch_add(&a.dctl->comp_tail, (uint64_t)1,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  write_completion_at(a, pos, req_id, status, data);
}

// Appends `nt` tiles of slot `slot` to the global tile sequence (caller
// holds the drain lock).  Returns false if the tile map has no room within
// the wait bound.
__device__ bool publish_tiles_locked(KArgsC& a, uint32_t slot, uint32_t nt) {
  uint64_t t0 = now_ticks();
  uint64_t pub = ld_dev_acq(&a.dctl->tiles_pub);
  while (pub + nt > ld_dev_acq(&a.dctl->tiles_done) + kTileMapCap / 2) {
    if (now_ticks() - t0 > a.wait_ticks) return false;
    backoff_sleep(2);
  }
  a.slots[slot].tile_base = pub;
  a.slots[slot].ntiles = nt;
  for (uint32_t t = 0; t < nt; ++t) a.tile2slot[(pub + t) & (kTileMapCap - 1)] = slot;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  st_dev_rel(&a.dctl->tiles_pub, pub + nt);
  return true;
}

__device__ __forceinline__ bool lock_drain(KArgsC& a, bool bounded) {
  uint64_t t0 = now_ticks();
  for (;;) {
    uint32_t z = 0;
    if (ld_dev(&a.dctl->drain_lock) == 0 && cas_dev(&a.dctl->drain_lock, z, 1u)) return true;
    if (!bounded) return false;
    if (now_ticks() - t0 > a.wait_ticks) return false;
    backoff_sleep(1);
  }
}

__device__ void unlock_drain(KArgsC& a) { st_dev_rel(&a.dctl->drain_lock, 0u); }

// Pipeline stages small enough to run where the previous stage finished:
// the workgroup that completes a message's last tile runs the next stage
// itself (no publication, no drain lock, no second claim) when that stage
// has at most this many work tiles.
constexpr uint32_t kInlineStageTiles = 16;

// Forwards the finished reply in `slot` to the next actor of its pipeline:
// the slot's descriptor becomes the next stage's (input = this reply).
// Returns true if the caller's workgroup is to run that stage inline;
// otherwise the stage is published for any workgroup, or (next actor gone,
// no room) the request is completed with an error.  Thread-level, drain
// kernel only.
CAF_RARE bool forward_reply(KArgsC& a, uint32_t slot) {
  const Desc d = a.slots[slot].d;
  const uint32_t hop = d.hop_actor[0];
  const uint32_t actor = (hop & 0xFFFFu) - 1u;
  const uint16_t behavior = (uint16_t)(hop >> 16);
  if (!actor_alive(a.hctl, actor)) {
    write_completion(a, d.req_id, CAF_E_QUIT, nullptr);
    return false;
  }
  Desc nd = d;
  nd.actor = actor;
  nd.behavior = behavior;
  nd.in0 = d.out;
  nd.in1 = 0;
  nd.out = d.hop_out[0];
  nd.hop_actor[0] = d.hop_actor[1];
  nd.hop_out[0] = d.hop_out[1];
  nd.hop_actor[1] = 0;
  nd.hop_out[1] = 0;
  const uint32_t rows = d.behavior == CAF_BHV_GEMM ? d.p.g.n : d.p.s.rows;
  const uint32_t cols = d.behavior == CAF_BHV_GEMM ? d.p.g.n : d.p.s.cols;
  for (int i = 0; i < 48; ++i) nd.p.raw[i] = 0;
  nd.p.s.rows = rows;
  nd.p.s.cols = cols;
  nd.flags = (uint16_t)(d.flags & DF_SEND);
  nd.tcfg = 0;
  a.slots[slot].d = nd;
  const uint32_t nt = desc_ntiles(nd);
  if (nt <= kInlineStageTiles) return true;
  bool ok = lock_drain(a, true);
  if (ok) {
    ok = publish_tiles_locked(a, slot, nt);
    unlock_drain(a);
  }
  if (!ok) write_completion(a, d.req_id, CAF_E_DEVICE, nullptr);
  return false;
}

// Completes (or forwards) the message in `slot` after its current stage:
// thread 0, once the workgroup's writes of the stage are done.  Returns true
// if the workgroup is to run the next stage inline.
__device__ __forceinline__ bool stage_done(KArgsC& a, const Desc& d, bool ring) {
  const uint32_t slot = d.slot;
  SlotState* ss = &a.sstate[slot];
  const int32_t st = ld_dev(&ss->status);
  if (ring && st == CAF_OK && d.hop_actor[0] != 0) return forward_reply(a, slot);
  if (!(d.flags & DF_NO_COMPLETE)) {
    st_dev(&ss->status, 0);
    const uint8_t* data = (d.flags & DF_INLINE_OUT) ? a.slots[slot].inline_out : nullptr;
    write_completion(a, d.req_id, st, data);
  }
  return false;
}

// Accounts `count` finished tiles of message `d` (thread 0, after the
// workgroup's tile work is complete).  The last tile of a message resets
// the slot's counters and completes or forwards it; returns true if the
// workgroup is to run the next pipeline stage inline.  A workgroup that ran
// every tile of the stage itself (a one-tile message, or a whole GEMM run)
// skips the shared count: no other workgroup's work has to be waited for.
__device__ __forceinline__ bool finish_tiles(KArgsC& a, const Desc& d, uint32_t ntiles,
                                             uint32_t count, bool ring) {
  const uint32_t slot = d.slot;
  SlotState* ss = &a.sstate[slot];
  bool cont = false;
  const bool whole = count == ntiles;
  // Tiles of a message finished by several workgroups: each releases its
  // part before counting it (on this chip a release writes back the
  // workgroup's L2, so it is not free).  A run that finishes the whole
  // message skips it: what follows -- the completion record (a system-scope
  // release), a publication of the next stage (an agent-scope release) or
  // that stage run by this workgroup -- orders the reply's data itself.
  if (!whole) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  const uint32_t prev =
      whole ? 0u
            : __hip_atomic_fetch_add(&ss->done, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (prev + count == ntiles) {
    if (!whole) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    st_dev(&ss->done, 0u);
    st_dev(&ss->decision, 0u);
    cont = stage_done(a, d, ring);
  }
  if (ring) __hip_atomic_fetch_add(&a.dctl->tiles_done, (uint64_t)count, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  return cont;
}
__device__ __forceinline__ bool finish_tile(KArgsC& a, const Desc& d, uint32_t ntiles, bool ring) {
  return finish_tiles(a, d, ntiles, 1u, ring);
}

// ---- behaviour dispatch -----------------------------------------------------

__device__ __forceinline__ void hash_step(KArgsC& a, const Desc& d) {
  if (threadIdx.x != 0) return;
  DevActor* act = &a.actors[d.actor];
  const uint64_t t0 = now_ticks();
  while (ld_dev_acq(&act->seq_done) != d.seq) {
    if (now_ticks() - t0 > a.wait_ticks) {
      st_dev(&a.sstate[d.slot].status, (int32_t)CAF_E_DEVICE);
      return;
    }
    backoff_sleep(1);
  }
  const uint64_t s = (ld_dev(&act->state) * 1000003ull) ^ d.p.h.x;
  st_dev(&act->state, s);
  uint64_t* io = reinterpret_cast<uint64_t*>(a.slots[d.slot].inline_out);
  io[0] = s;
  io[1] = 0;
  // A reply that does not travel in the completion record goes to the
  // message's output buffer (a caller-owned one, or the arena's); the
  // completion that follows releases it.
  if (!(d.flags & DF_INLINE_OUT) && d.out) *reinterpret_cast<uint64_t*>(d.out) = s;
  st_dev_rel(&act->seq_done, d.seq + 1u);
}

// LDS of a full variant: the largest work tile, two buffers of a bf16 GEMM
// slice at TE = 128, for slices of bk (with 64-deep slices it also holds the
// three stages of a wide bf16 tile).  The light variant only needs the drain
// scratch.
constexpr uint32_t smem_bytes(int bk) { return 2 * (2 * 128 * (bk + 8) * 2); }
static_assert(smem_bytes(kBf16SliceK) >= kWideSmemBytes, "wide bf16 tiles fit the full LDS");

// The square matrix tiles as calls, for the wide variant: inlined next to
// the wide tile their registers would spill.  A call costs a register save
// and restore per claimed run.
__device__ __noinline__ void gemm_bf16_tile_call(const uint16_t* A, const uint16_t* B, float* C,
                                                 uint32_t n, uint32_t te, uint32_t tile,
                                                 uint32_t count, uint16_t* smem) {
  if (te == 128) gemm_bf16_tile<128>(A, B, C, n, tile, count, smem);
  else gemm_bf16_tile<64>(A, B, C, n, tile, count, smem);
}
__device__ __noinline__ void gemm_f32_tile_call(const float* A, const float* B, float* C,
                                                uint32_t n, uint32_t te, uint32_t tile,
                                                uint32_t count, float* smem) {
  if (te == 128) gemm_f32_tile<128>(A, B, C, n, tile, count, smem);
  else gemm_f32_tile<64>(A, B, C, n, tile, count, smem);
}

// kFull = false compiles every behaviour except GEMM: without the matrix
// tiles the kernel needs far fewer registers and runs more waves per SIMD.
// One tile of every behaviour except GEMM (see run_tiles).
template <bool kFull>
__device__ __forceinline__ void run_tile(KArgsC& a, const Desc& d, uint32_t tile, uint8_t* smem,
                         uint32_t* lds_ctr) {
  switch (d.behavior) {
    case CAF_BHV_MANDELBROT:
      if (d.flags & DF_FP64) mandel_tile<double>(d, tile, 1u, lds_ctr);
      else mandel_tile<float>(d, tile, 1u, lds_ctr);
      break;
    case CAF_BHV_GEMM:
      // never reached: products run through run_tiles (one call site keeps
      // the tiles inlined), and a light launch does not drain GEMM messages
      if (threadIdx.x == 0) st_dev(&a.sstate[d.slot].status, (int32_t)CAF_E_DEVICE);
      break;
    case CAF_BHV_TANH:
      tanh_tile(reinterpret_cast<const float*>(d.in0), reinterpret_cast<float*>(d.out),
                (uint64_t)d.p.s.rows * d.p.s.cols, tile);
      break;
    case CAF_BHV_ROWSUM:
      rowsum_tile(reinterpret_cast<const float*>(d.in0), reinterpret_cast<float*>(d.out),
                  d.p.s.rows, d.p.s.cols, tile);
      break;
    case CAF_BHV_NOOP:
      echo_tile(d, a.slots[d.slot].inline_out);
      break;
    case CAF_BHV_HASHCHAIN:
      hash_step(a, d);
      break;
    case CAF_BHV_FAULT:
      if (threadIdx.x == 0) st_dev(&a.sstate[d.slot].status, (int32_t)CAF_E_FAULT);
      break;
    default:
      if (threadIdx.x == 0) st_dev(&a.sstate[d.slot].status, (int32_t)CAF_E_INVALID);
      break;
  }
}

// Tiles tile .. tile + count - 1 of one message (whole workgroup; for a GEMM
// these are work units, each `unit` output tiles).  The tiles of a GEMM run
// as one stream (the next tile's first slice loads while the current one
// finishes), those of a Mandelbrot message as one range of pixel blocks;
// other behaviours run tile by tile.
template <bool kFull, int kBk = kBf16SliceK, bool kWide = false>
__device__ __forceinline__ void run_tiles(KArgsC& a, const Desc& d, uint32_t tile,
                                          uint32_t count, uint8_t* smem, uint32_t* lds_ctr) {
  if constexpr (kWide) {
    if (d.behavior == CAF_BHV_GEMM) {
      // work units -> output tiles
      const uint32_t u = gemm_unit(d), all = gemm_tiles(d);
      const uint32_t t0 = tile * u;
      const uint32_t cnt = min(t0 + count * u, all) - t0;
      float* C = reinterpret_cast<float*>(d.out);
      if (d.flags & DF_BF16) {
        const uint16_t* A = reinterpret_cast<const uint16_t*>(d.in0);
        const uint16_t* B = reinterpret_cast<const uint16_t*>(d.in1);
        if (d.tcfg == 256) gemm_bf16_tile_wide(A, B, C, d.p.g.n, t0, cnt, (uint16_t*)smem);
        else gemm_bf16_tile_call(A, B, C, d.p.g.n, d.tcfg, t0, cnt, (uint16_t*)smem);
      } else {
        gemm_f32_tile_call(reinterpret_cast<const float*>(d.in0),
                           reinterpret_cast<const float*>(d.in1), C, d.p.g.n, d.tcfg, t0, cnt,
                           (float*)smem);
      }
      return;
    }
  } else if constexpr (kFull) {
    if (d.behavior == CAF_BHV_GEMM) {
      if (d.tcfg == 256) {  // wide tiles run in the wide variant only
        if (threadIdx.x == 0) st_dev(&a.sstate[d.slot].status, (int32_t)CAF_E_DEVICE);
        return;
      }
      // work units -> output tiles
      const uint32_t u = gemm_unit(d), all = gemm_tiles(d);
      const uint32_t t0 = tile * u;
      count = min(t0 + count * u, all) - t0;
      tile = t0;
      float* C = reinterpret_cast<float*>(d.out);
      if (d.flags & DF_BF16) {
        const uint16_t* A = reinterpret_cast<const uint16_t*>(d.in0);
        const uint16_t* B = reinterpret_cast<const uint16_t*>(d.in1);
        if (d.tcfg == 128)
          gemm_bf16_tile<128, kBk>(A, B, C, d.p.g.n, tile, count, (uint16_t*)smem);
        else gemm_bf16_tile<64, kBk>(A, B, C, d.p.g.n, tile, count, (uint16_t*)smem);
      } else {
        const float* A = reinterpret_cast<const float*>(d.in0);
        const float* B = reinterpret_cast<const float*>(d.in1);
        if (d.tcfg == 128) gemm_f32_tile<128>(A, B, C, d.p.g.n, tile, count, (float*)smem);
        else gemm_f32_tile<64>(A, B, C, d.p.g.n, tile, count, (float*)smem);
      }
      return;
    }
  }
  if (d.behavior == CAF_BHV_MANDELBROT) {
    if (d.flags & DF_FP64) mandel_tile<double>(d, tile, count, lds_ctr);
    else mandel_tile<float>(d, tile, count, lds_ctr);
    return;
  }
  for (uint32_t i = 0; i < count; ++i) {
    if (i) __syncthreads();
    run_tile<kFull>(a, d, tile + i, smem, lds_ctr);
  }
}

// A pipeline stage (row-wise tanh or row sum of a float matrix) run inline
// by the workgroup that finished the previous stage: every tile in turn.
// `s_flag` is workgroup-shared scratch.  Whole workgroup.
__device__ __forceinline__ void run_inline_stages(KArgsC& a, uint32_t slot, uint32_t* s_flag) {
  for (;;) {
    __syncthreads();
    Desc d;
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&a.slots[slot].d);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&d);
#pragma unroll
      for (int q = 0; q < (int)(sizeof(Desc) / 4); ++q)
        dst[q] = __builtin_amdgcn_readfirstlane(src[q]);
    }
    const uint32_t nt = desc_ntiles(d);
    for (uint32_t tt = 0; tt < nt; ++tt) {
      if (ld_dev(&a.sstate[slot].status) == CAF_OK) {
        if (d.behavior == CAF_BHV_TANH)
          tanh_tile(reinterpret_cast<const float*>(d.in0), reinterpret_cast<float*>(d.out),
                    (uint64_t)d.p.s.rows * d.p.s.cols, tt);
        else if (d.behavior == CAF_BHV_ROWSUM)
          rowsum_tile(reinterpret_cast<const float*>(d.in0), reinterpret_cast<float*>(d.out),
                      d.p.s.rows, d.p.s.cols, tt);
        else if (threadIdx.x == 0)
          st_dev(&a.sstate[slot].status, (int32_t)CAF_E_INVALID);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      *s_flag = stage_done(a, d, true) ? 1u : 0u;
    }
    __syncthreads();
    if (!*s_flag) break;
  }
}

constexpr uint32_t kSmemBytes = smem_bytes(kBf16SliceK);

// ---- one launch per message -------------------------------------------------

template <bool kFull>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
plain_kernel(KArgs, Desc d, uint32_t ntiles) {
  KArgsC& a = kargs();
  __shared__ __align__(16) uint8_t smem[kSmemBytes];
  __shared__ uint32_t s_dec;
  __shared__ uint32_t s_ctr;
  const uint32_t slot = d.slot;
  SlotState* ss = &a.sstate[slot];
  if (threadIdx.x == 0) {
    // All workgroups of the message agree on one reading of the actor's
    // alive flag: the first to arrive decides.
    uint32_t dec = ld_dev_acq(&ss->decision);
    if (dec == 0) {
      const uint32_t v = actor_alive(a.hctl, d.actor) ? 1u : 2u;
      uint32_t z = 0;
      dec = cas_dev(&ss->decision, z, v) ? v : z;
    }
    if (dec == 2) {
      int32_t ok = 0;
      __hip_atomic_compare_exchange_strong(&ss->status, &ok, (int32_t)CAF_E_QUIT,
                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    }
    s_dec = (dec == 1 && ld_dev(&ss->status) == CAF_OK) ? 1u : 0u;
  }
  __syncthreads();
  if (s_dec) run_tiles<kFull>(a, d, blockIdx.x, 1u, smem, &s_ctr);
  __syncthreads();
  if (threadIdx.x == 0) finish_tile(a, d, ntiles, false);
}

// ---- the mailbox drain ----------------------------------------------------

// Sort key of a drained entry (smaller keys are laid out first): the
// behaviour, and under CAF_GROUP_LPT the product size too, largest first.
// CAF_GROUP_KIND groups by behaviour only and keeps the mailbox order of the
// products: sorting a pass largest first leaves its end to the smallest
// products, whose fixed per-product costs weigh most, while the next pass
// starts with large ones again.
__device__ __forceinline__ uint32_t group_key(const Desc& e, uint32_t grouping) {
  switch (e.behavior) {
    case CAF_BHV_GEMM: {
      if (grouping != CAF_GROUP_LPT) return 0u;
      const uint32_t n = e.p.g.n;
      return n >= 512 ? 0u : n >= 256 ? 1u : n >= 128 ? 2u : n >= 64 ? 3u : 4u;
    }
    case CAF_BHV_MANDELBROT: return 5u;
    case CAF_BHV_TANH: return 6u;
    case CAF_BHV_ROWSUM: return 7u;
    default: return 8u;
  }
}
constexpr uint32_t kKeys = 9;

struct DrainLds {
  uint32_t slot[kMaxBatch];
  uint32_t nt[kMaxBatch];
  uint32_t scan[kMaxBatch];  // tile counts by position, then their exclusive prefix
  uint16_t pos[kMaxBatch];
  uint8_t key[kMaxBatch];
  uint8_t dead[kMaxBatch];
  // hash-chain entries the drain runs itself: actor + 1 (0: not one), the
  // new state, and the list of entries run
  uint16_t hactor[kMaxBatch];
  uint64_t hx[kMaxBatch];
  uint16_t hidx[kMaxBatch];
  // echo entries with inline input and reply, answered by the drain itself
  uint8_t inl[kMaxBatch];
  uint32_t nh;
  uint32_t any_hash;  // some entry is one
  uint32_t any_echo;  // some entry is an inline echo
  uint64_t hpos;
  uint32_t first_bad;  // light launch: first entry it cannot run
  uint32_t any_dead;   // some entry's actor looked dead in the snapshot
  uint32_t alive[kAliveWords];
  uint32_t hist[kKeys];
  uint32_t running[kKeys];
  uint32_t wave_cnt[4][kKeys];
  uint32_t wave_sum[4];
  uint64_t d, cnt, pub, done;
  uint32_t total;
  // set by a sentinel before its drain pass: the launch may retire if the
  // pass finds the mailbox empty and the drained count still equal to this
  // (checked under the drain lock)
  uint32_t retire_ok;
  uint64_t retire_drained;
};
static_assert(sizeof(DrainLds) <= smem_bytes(32), "drain scratch fits every tile LDS");
constexpr uint32_t kSmemLight = (sizeof(DrainLds) + 15u) / 16u * 16u;

// In-place exclusive prefix sum of v[0..count), count <= 1024, whole workgroup.
__device__ uint32_t block_exclusive_scan(uint32_t* v, uint32_t count, uint32_t* wave_sum) {
  const uint32_t t = threadIdx.x, lane = lane_id(), w = wave_id();
  uint32_t loc[4];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t idx = t * 4 + i;
    loc[i] = idx < count ? v[idx] : 0u;
    s += loc[i];
  }
  uint32_t incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off);
    if (lane >= (uint32_t)off) incl += o;
  }
  if (lane == 63) wave_sum[w] = incl;
  __syncthreads();
  uint32_t wbase = 0, total = 0;
  for (uint32_t i = 0; i < 4; ++i) {
    if (i < w) wbase += wave_sum[i];
    total += wave_sum[i];
  }
  uint32_t run = wbase + incl - s;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t idx = t * 4 + i;
    if (idx < count) v[idx] = run;
    run += loc[i];
  }
  __syncthreads();
  return total;
}

// Drain ahead when fewer than this many published tiles per workgroup are
// left unclaimed (and the mailbox holds a backlog).
constexpr uint64_t kDrainAheadPerWg = 4;

// Largest drain pass whose inline echoes the drain answers itself.
constexpr uint32_t kDrainEchoMax = 4;

// A workgroup's reservation of claimed tile indices (see "claiming work
// tiles" below).
struct Claim {
  uint64_t next = 0, end = 0;  // tiles [next, end) are this workgroup's
  bool own = false;  // published by this workgroup's own drain pass
};

// Returns the published count it read (0 if it reserved nothing).  pub and
// cur: the published count and the claim cursor, just read.
__device__ __forceinline__ uint64_t reserve(KArgsC& a, Claim& c, uint64_t pub, uint64_t cur) {
  if (cur >= pub) return 0;
  // Guided self-scheduling: large chunks while plenty is published.  The
  // full variant takes twice as large chunks: a run that covers a whole
  // product skips its release, while escape-time tiles, whose cost is not
  // known in advance, need the smaller chunks to end a batch evenly.
  const uint64_t avail = pub - cur, g2 = (a.full ? 1ull : 2ull) * a.grid;
  const uint64_t k = avail >= 16 * g2 ? 16 : avail >= 8 * g2 ? 8 : avail >= 4 * g2 ? 4
                     : avail >= 2 * g2 ? 2 : 1;
  c.next = __hip_atomic_fetch_add(&a.dctl->tiles_claimed, k, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  c.end = c.next + k;
  return pub;
}

// Stateful hash-chain entries of entries [0, cnt) run here, in mailbox
// order, while the drain lock is held: the state update is a few
// instructions, and done by the drainer it needs no hand-off between
// workgroups (a tile waiting for its predecessor's sequence number takes a
// device round trip per step).  Per actor, entries run while their sequence
// numbers continue the actor's; from the first that does not (an earlier
// entry of the actor went the tile way) the rest go the tile way too, where
// they wait their turn.  Entries run here get no tiles (nt = 0).  Wave 0
// finds each actor's entries 64 at a time with ballots; lane 0 applies them.
__device__ void run_hash_entries_locked(KArgsC& a, DrainLds& L, uint32_t cnt) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t nh = 0;  // lane 0's count
  if (!L.any_hash) cnt = 0;
  for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
    for (;;) {
      const uint32_t j = c0 + lane;
      const uint64_t m = __ballot(j < cnt && L.hactor[j] != 0);
      if (m == 0) break;
      // the first entry not handled yet starts its actor's chain
      const uint32_t x1 = L.hactor[c0 + (uint32_t)__builtin_ctzll(m)];
      DevActor* act = &a.actors[x1 - 1u];
      uint32_t next = 0;
      uint64_t st = 0;
      bool ok = true, any = false;
      if (lane == 0) {
        next = ld_dev_acq(&act->seq_done);
        st = ld_dev(&act->state);
      }
      for (uint32_t d0 = c0; d0 < cnt; d0 += 64) {
        const uint32_t jj = d0 + lane;
        const bool mine = jj < cnt && L.hactor[jj] == x1;
        uint64_t mm = __ballot(mine);
        if (mine) L.hactor[jj] = 0;
        if (lane == 0) {
          while (mm) {
            const uint32_t k = d0 + (uint32_t)__builtin_ctzll(mm);
            mm &= mm - 1;
            const Desc& e = a.slots[L.slot[k]].d;  // written by this workgroup this pass
            if (!ok || e.seq != next) {
              ok = false;
              continue;
            }
            st = (st * 1000003ull) ^ e.p.h.x;
            L.hx[k] = st;
            L.hidx[nh++] = (uint16_t)k;
            L.nt[k] = 0;
            ++next;
            any = true;
          }
        }
      }
      if (lane == 0 && any) {
        st_dev(&act->state, st);
        st_dev_rel(&act->seq_done, next);
      }
    }
  }
  if (lane == 0) L.nh = nh;
}

// The replies of the entries the drain answers itself -- the hash-chain
// entries run by run_hash_entries_locked and the inline echo entries -- one
// completion position reservation, then the records in parallel (whole
// workgroup).
__device__ void complete_hash_entries(KArgsC& a, DrainLds& L) {
  const uint32_t t = threadIdx.x;
  const uint32_t nh = L.nh;
  if (nh == 0) return;
  if (t == 0)
    L.hpos = __hip_atomic_fetch_add(&a.dctl->comp_tail, (uint64_t)nh, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (uint32_t j = t; j < nh; j += kThreads) {
    const uint32_t i = L.hidx[j];
    const Desc& e = a.slots[L.slot[i]].d;  // written by this workgroup this pass
    uint64_t v[2] = {L.hx[i], 0ull};
    // an inline echo replies with its inline input (at most four int32)
    if (L.inl[i]) __builtin_memcpy(v, e.p.raw, sizeof v);
    write_completion_at(a, L.hpos + j, e.req_id, CAF_OK, reinterpret_cast<const uint8_t*>(v));
  }
}

// Drains one batch from the mailbox (whole workgroup; the caller holds the
// drain lock, which is released here).  Returns true if anything was drained.
__device__ __forceinline__ bool drain_once_body(KArgsC& a, DrainLds& L, bool may_claim,
                                                Claim& cl) {
  const uint32_t t = threadIdx.x;
  // One PCIe round trip: the ring tail, the stop flag and a snapshot of the
  // actors' alive bits are read together (the snapshot by the second wave,
  // so that thread 0 does not wait for it before issuing its own loads).
  // The snapshot is not ordered after the tail read, so a bit the host set
  // just before publishing an entry can be missing from it; entries that
  // look dead are checked again below.
  static_assert(kAliveWords <= 64, "one wave reads the alive words");
  if (t >= 64 && t < 64 + kAliveWords) L.alive[t - 64] = ld_sys(&a.hctl->alive[t - 64]);
  if (t == 0) L.any_dead = 0;
  if (t == 0) L.any_hash = 0;
  if (t == 0) L.any_echo = 0;
  if (t == 0) {
    // All five loads are in flight together; one system-scope acquire fence
    // after them orders the entry reads below after the tail (each acquire
    // load on its own would wait for its own round trip).
    const uint32_t stop = ld_sys(&a.hctl->stop);
    const uint64_t tail = ld_sys(&a.hctl->tail);
    const uint64_t d = ld_dev(&a.dctl->drained);
    const uint64_t pubv = ld_dev(&a.dctl->tiles_pub);
    const uint64_t done = ld_dev(&a.dctl->tiles_done);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const uint64_t avail = tail - d;
    L.d = d;
    L.cnt = avail < a.max_batch ? avail : a.max_batch;
    // Lets idle workgroups help while a backlog remains (relaxed: a hint).
    st_dev(&a.dctl->backlog, avail > a.max_batch ? 1u : 0u);
    L.pub = pubv;
    L.done = done;
    if (stop) st_dev(&a.dctl->stop_seen, 1u);
  }
  if (t < kKeys) L.hist[t] = 0;
  if (t == 0) L.first_bad = ~0u;
  __syncthreads();
  uint32_t cnt = (uint32_t)L.cnt;
  if (cnt == 0) {
    if (t == 0) {
      // An idle batched launch retires here, holding the drain lock: no other
      // pass can be publishing, and the tail was just read.  Every workgroup
      // of it leaves once it holds no work (claimed tiles are finished
      // first), and the host starts a new launch when messages arrive.
      if (L.retire_ok && L.d == L.retire_drained && ld_dev(&a.dctl->tiles_claimed) >= L.pub) {
        const uint32_t par = a.gen & 1u;
        st_dev(&a.dctl->retiring[par], a.gen);
        st_sys_rel(&a.hctl->retiring[par], a.gen);
      }
      unlock_drain(a);
    }
    return false;
  }
  // Copy the entries into their device slots.
  for (uint32_t i = t; i < cnt; i += kThreads) {
    // Plain 16-byte loads (eight PCIe reads per entry): the host wrote the
    // entry before the tail, and the acquire fence after the tail read
    // dropped any cached copy of it.
    const auto src = global_ptr(reinterpret_cast<const uint32_t*>(&a.hring[(L.d + i) % a.cap]));
    struct Raw {
      uint4 q[sizeof(Desc) / 16];
    } raw;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Desc) / 16); ++q) raw.q[q] = load_global<uint4>(src + 4 * q);
    const Desc e = __builtin_bit_cast(Desc, raw);
    const bool alive = (L.alive[e.actor >> 5] >> (e.actor & 31)) & 1u;
    const uint32_t slot = e.slot;
    a.slots[slot].d = e;
    L.slot[i] = slot;
    L.nt[i] = alive ? desc_ntiles(e) : 0u;
    L.dead[i] = alive ? 0 : 1;
    if (!alive) L.any_dead = 1;
    L.key[i] = (uint8_t)(a.grouping != CAF_GROUP_FIFO ? group_key(e, a.grouping) : 0u);
    const bool hash_here = alive && e.behavior == CAF_BHV_HASHCHAIN && e.hop_actor[0] == 0 &&
                           (e.flags & (DF_INLINE_OUT | DF_SEND)) != 0;
    L.hactor[i] = hash_here ? (uint16_t)(e.actor + 1u) : (uint16_t)0;
    if (hash_here) L.any_hash = 1;
    // An echo whose input and reply both travel inline (a ping-pong
    // message) in a pass of at most kDrainEchoMax entries: the drain answers
    // it itself, with no tile, publication or claim, which is what a reply
    // that is waited for needs.  In larger passes the echoes go the tile
    // way, where many workgroups write their replies while the next pass
    // drains.  An echo keeps no state, so answering it here instead of as a
    // tile changes no observable order.
    const bool echo_here = alive && L.cnt <= kDrainEchoMax && e.behavior == CAF_BHV_NOOP &&
                           e.hop_actor[0] == 0 &&
                           (e.flags & DF_INLINE_IN) != 0 &&
                           (e.flags & (DF_INLINE_OUT | DF_SEND)) != 0;
    L.inl[i] = echo_here ? 1u : 0u;
    if (echo_here) {
      L.nt[i] = 0;
      L.any_echo = 1;
    }
    if (!a.full && e.behavior == CAF_BHV_GEMM) atomicMin(&L.first_bad, i);
  }
  __syncthreads();
  if (L.any_dead) {
    // Re-read the alive word of each entry that looked dead; this read is
    // issued after the tail acquire (the barrier above orders it), so a
    // spawn that happened before the entry was published is visible.
    for (uint32_t i = t; i < cnt; i += kThreads) {
      if (!L.dead[i]) continue;
      const Desc& e = a.slots[L.slot[i]].d;
      if ((ld_sys(&a.hctl->alive[e.actor >> 5]) >> (e.actor & 31)) & 1u) {
        L.dead[i] = 0;
        L.nt[i] = desc_ntiles(e);
      }
    }
    __syncthreads();
  }
  if (L.first_bad < cnt) {
    // A light launch drains only the entries before the first GEMM message
    // and, if that is the head of the mailbox, retires so that the host
    // starts a full launch.
    cnt = L.first_bad;
    if (cnt == 0) {
      if (t == 0) {
        st_dev(&a.dctl->retiring[a.gen & 1u], a.gen);
        st_sys_rel(&a.hctl->retiring[a.gen & 1u], a.gen);
        unlock_drain(a);
      }
      return false;
    }
  }
  // Flow control: keep the tile map ahead of the slowest reader by half its size.
  const uint64_t room = kTileMapCap / 2 - (L.pub - L.done);
  uint32_t total;
  if (cnt == 1) {
    // A single entry (the common case at low load): no scan, no grouping.
    if (L.nt[0] > room) {
      if (t == 0) unlock_drain(a);
      return false;
    }
    if (t < 64) run_hash_entries_locked(a, L, 1);
    if (t == 0) {
      L.pos[0] = 0;
      L.scan[0] = 0;
    }
    __syncthreads();
    total = L.nt[0];
  } else {
    for (uint32_t i = t; i < cnt; i += kThreads) L.scan[i] = L.nt[i];
    __syncthreads();
    total = block_exclusive_scan(L.scan, cnt, L.wave_sum);
    if (total > room) {
      if (t == 0) {
        uint32_t c = 0;
        while (c < cnt && (uint64_t)L.scan[c] + L.nt[c] <= room) ++c;
        L.cnt = c;
      }
      __syncthreads();
      cnt = (uint32_t)L.cnt;
      if (cnt == 0) {
        if (t == 0) unlock_drain(a);
        return false;
      }
    }
    if (t < 64) run_hash_entries_locked(a, L, cnt);
    __syncthreads();
    // Grouping: stable counting sort of the batch by key.
    if (a.grouping != CAF_GROUP_FIFO) {
      for (uint32_t i = t; i < cnt; i += kThreads) atomicAdd(&L.hist[L.key[i]], 1u);
      __syncthreads();
      if (t == 0) {
        uint32_t run = 0;
        for (uint32_t k = 0; k < kKeys; ++k) {
          L.running[k] = run;
          run += L.hist[k];
        }
      }
      __syncthreads();
      const uint32_t lane = lane_id(), w = wave_id();
      const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      for (uint32_t c0 = 0; c0 < cnt; c0 += kThreads) {
        const uint32_t i = c0 + t;
        const bool valid = i < cnt;
        const uint32_t k = valid ? L.key[i] : kKeys;
        uint32_t rank = 0;
        for (uint32_t kk = 0; kk < kKeys; ++kk) {
          const uint64_t m = __ballot(valid && k == kk);
          if (k == kk) rank = __popcll(m & lt_mask);
          if (lane == 0) L.wave_cnt[w][kk] = __popcll(m);
        }
        __syncthreads();
        uint32_t off = 0;
        if (valid) {
          off = L.running[k];
          for (uint32_t ww = 0; ww < w; ++ww) off += L.wave_cnt[ww][k];
        }
        __syncthreads();
        if (t < kKeys)
          for (uint32_t ww = 0; ww < 4; ++ww) L.running[t] += L.wave_cnt[ww][t];
        if (valid) L.pos[i] = (uint16_t)(off + rank);
        __syncthreads();
      }
    } else {
      for (uint32_t i = t; i < cnt; i += kThreads) L.pos[i] = (uint16_t)i;
    }
    __syncthreads();
    // Prefix of tile counts in work order.
    for (uint32_t i = t; i < cnt; i += kThreads) L.scan[L.pos[i]] = L.nt[i];
    __syncthreads();
    total = block_exclusive_scan(L.scan, cnt, L.wave_sum);
  }  // cnt > 1
  const uint64_t pub = L.pub;
  for (uint32_t i = t; i < cnt; i += kThreads) {
    const uint32_t slot = L.slot[i], nt = L.nt[i];
    const uint64_t base = pub + L.scan[L.pos[i]];
    a.slots[slot].tile_base = base;
    a.slots[slot].ntiles = nt;
    for (uint32_t k = 0; k < nt; ++k) a.tile2slot[(base + k) & (kTileMapCap - 1)] = slot;
    if (L.dead[i]) write_completion(a, a.slots[slot].d.req_id, CAF_E_QUIT, nullptr);
  }
  if (L.any_echo) {
    // the inline echoes of the entries drained in this pass join the list
    // of replies the drain writes itself
    __syncthreads();
    for (uint32_t i = t; i < cnt; i += kThreads)
      if (L.inl[i]) L.hidx[atomicAdd(&L.nh, 1u)] = (uint16_t)i;
    __syncthreads();
  }
  complete_hash_entries(a, L);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (t == 0) {
    // The fence and barrier above release the slots and tile map written by
    // every thread, so the tiles are published first, without another fence.
    // The unlock releases the drained counts: the host copy must never move
    // backwards, so it lands before the next holder can write its own.
    // The drainer takes one index before the tiles become visible, so it
    // runs the first of them itself (a one-message pass is usually a reply
    // waited for, and the slots and tile map it just wrote are in its L2);
    // an index beyond them is an ordinary reservation.
    if (total && may_claim) {
      cl.next = __hip_atomic_fetch_add(&a.dctl->tiles_claimed, (uint64_t)1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
      cl.end = cl.next + 1;
      cl.own = cl.next >= pub && cl.next < pub + total;
    }
    st_dev(&a.dctl->tiles_pub, pub + total);
    st_dev(&a.dctl->drained, L.d + cnt);
    st_sys(&a.hctl->drained, L.d + cnt);
    unlock_drain(a);
  }
  return true;
}

// The full variant keeps the drain out of line (its tile loop already needs
// most registers); the light variant inlines it, so that the whole kernel is
// allocated under its five-waves-per-SIMD register budget.
// (Its result comes back by value, so the caller's reservation stays in
// registers.)
struct DrainOut {
  uint64_t next, end;
  bool own, got;
};
CAF_RARE DrainOut drain_once_outlined(KArgsC& a, DrainLds& L, bool may_claim) {
  Claim cl;
  const bool got = drain_once_body(a, L, may_claim, cl);
  return DrainOut{cl.next, cl.end, cl.own, got};
}

template <bool kFull>
__device__ __forceinline__ bool drain_once(KArgsC& a, DrainLds& L, Claim& c) {
  // thread 0 may come back with a reservation of the tiles just published
  if constexpr (kFull) {
    const DrainOut r = drain_once_outlined(a, L, c.next == c.end);
    if (r.end > r.next) {
      c.next = r.next;
      c.end = r.end;
      c.own = r.own;
    }
    return r.got;
  } else {
    Claim cl;
    const bool got = drain_once_body(a, L, c.next == c.end, cl);
    if (cl.end > cl.next) c = cl;
    return got;
  }
}

// ---- claiming work tiles ----------------------------------------------
//
// A workgroup reserves tiles of the global sequence with one fetch_add on
// the claim cursor -- never a retried compare-and-swap, whose throughput
// collapses when hundreds of workgroups contend -- and only when the cursor
// is below the published count.  Racing workgroups can still overshoot:
// an index at or beyond the published count is then a reservation that the
// next publication fills (publications start at the published count, so the
// next published tiles are exactly the reserved ones).  Before anyone
// leaves (retire or stop), holders of unfilled reservations publish filler
// tiles for every reserved index, so no index is ever abandoned and no
// message tile is ever skipped.

// Publishes filler tiles for every reserved but unpublished index (caller
// holds the drain lock).
__device__ void fill_reservations_locked(KArgsC& a) {
  const uint64_t pub = ld_dev_acq(&a.dctl->tiles_pub);
  const uint64_t cl = ld_dev(&a.dctl->tiles_claimed);
  if (cl <= pub) return;
  for (uint64_t i = pub; i < cl; ++i) a.tile2slot[i & (kTileMapCap - 1)] = kNopTile;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  st_dev_rel(&a.dctl->tiles_pub, cl);
}

enum : uint32_t { CMD_IDLE = 0, CMD_TILE = 1, CMD_DRAIN = 2 };
constexpr uint32_t kSentinels = 16;

template <bool kFull, int kBk = kBf16SliceK, bool kWide = false>
__device__ __forceinline__ void drain_body(KArgsC& a) {
  __shared__ __align__(16) uint8_t smem[kFull ? smem_bytes(kBk) : kSmemLight];
  __shared__ __align__(16) DevSlot s_slot;
  __shared__ uint32_t s_cmd, s_exit, s_ctr, s_k, s_nop, s_cont;
  __shared__ int32_t s_status;
  __shared__ uint64_t s_g;
  // sentinel: the published and drained counts last seen, and since when
  // they have not moved (thread 0; kept in LDS, not in registers)
  __shared__ uint64_t s_seen_drained, s_still_since;
  __shared__ uint32_t s_retire_ok;
  const uint32_t t = threadIdx.x;
  uint64_t last_work = now_ticks();
  // At the start of a launch only the sentinels try the drain lock: every
  // workgroup trying it at once is a storm of compare-and-swaps (each with
  // its fences) that delays the first drain pass by microseconds.
  uint32_t idle_rounds = blockIdx.x < kSentinels ? 0u : 1u;
  Claim c;  // thread 0's reservation
  if (t == 0) {
    s_seen_drained = ~0ull;
    s_still_since = last_work;
    s_retire_ok = 0;
  }
  for (;;) {
    if (t == 0) {
      uint32_t cmd = CMD_IDLE;
      uint64_t pub = 0;
      if (c.next == c.end) {
        const uint64_t pub0 = ld_dev(&a.dctl->tiles_pub);
        const uint64_t cur0 = ld_dev(&a.dctl->tiles_claimed);
        // Drain ahead: while the mailbox holds more than one pass and the
        // published tiles nobody has claimed yet run low, this workgroup
        // takes the next pass now (one attempt at the lock), so that the
        // others are not left without tiles while it is drained.
        if (cur0 + kDrainAheadPerWg * a.grid > pub0 && ld_dev(&a.dctl->backlog) != 0 &&
            lock_drain(a, false))
          cmd = CMD_DRAIN;
        else
          pub = reserve(a, c, pub0, cur0);
      }
      if (c.next < c.end && c.own) {
        // An index of this workgroup's own drain pass: published, its slot
        // and tile map entry are this workgroup's writes, and the pass's
        // system-scope acquire already covers the message's data.
        s_g = c.next;
        s_k = (uint32_t)(c.end - c.next);
        c.next = c.end;
        c.own = false;
        cmd = CMD_TILE;
      } else if (c.next < c.end) {
        // the count read while reserving usually covers the new indices
        if (c.next >= pub) pub = ld_dev(&a.dctl->tiles_pub);
        if (c.next < pub) {
          const uint64_t n = (c.end < pub ? c.end : pub) - c.next;
          s_g = c.next;
          s_k = (uint32_t)n;
          c.next += n;
          cmd = CMD_TILE;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      // Draining an empty mailbox still holds the lock for a host round
      // trip, so idle workgroups do not all poll it: the sentinels do, a
      // workgroup that just finished work tries once, and so does one
      // waiting for its reserved index to be published; everyone helps
      // while the last pass left a backlog.
      const bool may_drain = blockIdx.x < kSentinels || idle_rounds == 0 || c.next < c.end ||
                             ld_dev(&a.dctl->backlog) != 0;
      if (cmd == CMD_IDLE && may_drain && lock_drain(a, false)) cmd = CMD_DRAIN;
      s_cmd = cmd;
    }
    __syncthreads();
    const uint32_t cmd = s_cmd;
    if (cmd == CMD_TILE) {
      const uint64_t g0 = s_g;
      const uint32_t nk = s_k;
      for (uint32_t j = 0; j < nk;) {
        const uint64_t g = g0 + j;
        // Thread 0 copies the message's slot while the second wave's first
        // lane reads its status, both after the same tile-map lookup: one
        // memory round trip fewer per run.
        if (t == 0 || t == 64) {
          const uint32_t slot = ld_dev(&a.tile2slot[g & (kTileMapCap - 1)]);
          if (t == 0) {
            s_nop = slot == kNopTile;
            if (!s_nop) s_slot = a.slots[slot];
          } else {
            s_status = slot == kNopTile ? (int32_t)CAF_OK : ld_dev(&a.sstate[slot].status);
          }
        }
        __syncthreads();
        if (s_nop) {  // a filler tile: nothing to do
          if (t == 0)
            __hip_atomic_fetch_add(&a.dctl->tiles_done, (uint64_t)1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          __syncthreads();
          ++j;
          continue;
        }
        // The descriptor is the same for every lane: move it to scalar
        // registers so the tile code sees uniform parameters.
        Desc d;
        {
          const uint32_t* src = reinterpret_cast<const uint32_t*>(&s_slot.d);
          uint32_t* dst = reinterpret_cast<uint32_t*>(&d);
#pragma unroll
          for (int q = 0; q < (int)(sizeof(Desc) / 4); ++q)
            dst[q] = __builtin_amdgcn_readfirstlane(src[q]);
        }
        const uint32_t ntiles = __builtin_amdgcn_readfirstlane(s_slot.ntiles);
        const uint32_t tile = __builtin_amdgcn_readfirstlane((uint32_t)(g - s_slot.tile_base));
        // The claimed indices that follow and still belong to this GEMM or
        // Mandelbrot message run together, with one lookup and one
        // completion count.
        const bool runs = (kFull && d.behavior == CAF_BHV_GEMM) || d.behavior == CAF_BHV_MANDELBROT;
        const uint32_t run = runs ? min(nk - j, ntiles - tile) : 1u;
        // A failed tile stops the message's other tiles; a one-tile message
        // cannot have failed before its tile runs.
        if (ntiles == 1 || s_status == CAF_OK)
          run_tiles<kFull, kBk, kWide>(a, d, tile, run, smem, &s_ctr);
        __syncthreads();
        if (t == 0) s_cont = finish_tiles(a, d, ntiles, run, true) ? 1u : 0u;
        __syncthreads();
        if (s_cont) run_inline_stages(a, d.slot, &s_cont);
        j += run;
      }
      last_work = now_ticks();
      idle_rounds = 0;
      continue;
    }
    if (cmd == CMD_DRAIN) {
      DrainLds& L = *reinterpret_cast<DrainLds*>(smem);
      if (t == 0) {
        L.retire_ok = s_retire_ok;
        L.retire_drained = s_seen_drained;
      }
      const bool got = drain_once<kFull>(a, L, c);
      __syncthreads();
      if (got) {
        last_work = now_ticks();
        idle_rounds = 0;
        continue;
      }
    }
    if (t == 0) {
      uint32_t ex = 0;
      const uint32_t par = a.gen & 1u;
      const bool holding = c.next < c.end;  // reserved, not yet published
      const bool leaving =
          ld_dev(&a.dctl->stop_seen) || ld_dev(&a.dctl->retiring[par]) == a.gen;
      if (holding) {
        // Nobody may leave an index unexecuted: before this launch goes (or
        // once this workgroup has idled as long as a launch may linger),
        // fill the outstanding reservations with filler tiles.  One lock
        // attempt per round: spinning on it here would stop this workgroup
        // from noticing that its index has been published meanwhile.
        if ((leaving || now_ticks() - last_work > a.idle_ticks) && lock_drain(a, false)) {
          fill_reservations_locked(a);
          unlock_drain(a);
        }
      } else if (leaving) {
        ex = 1;
      } else if (blockIdx.x < kSentinels) {
        // The system counts as idle once no drain pass has taken a message
        // for the linger time while this sentinel had no work (its own last
        // work says nothing about the others'; every published tile comes
        // from such a pass, except fillers, which carry no work).  Then its
        // next drain pass retires the launch if it finds the mailbox empty
        // and the drained count unchanged (batched mode lingers a few tens
        // of microseconds, persistent mode much longer).
        const uint64_t drv = ld_dev(&a.dctl->drained);
        const uint64_t now = now_ticks();
        if (drv != s_seen_drained || idle_rounds == 0) {
          s_seen_drained = drv;
          s_still_since = now;
          s_retire_ok = 0;
        } else {
          s_retire_ok = now - s_still_since > a.idle_ticks &&
                        ld_dev(&a.dctl->tiles_claimed) >= ld_dev(&a.dctl->tiles_pub) ? 1u : 0u;
        }
      }
      s_exit = ex;
      if (!ex) {
        // A few sentinel workgroups poll with a short back-off (reply
        // latency), and so does a workgroup holding a reserved index (the
        // next published tile is its to run); the rest back off further.
        const uint32_t cap = (blockIdx.x < kSentinels || holding) ? 1u : 8u;
        idle_rounds = idle_rounds < cap ? idle_rounds + 1 : cap;
        backoff_sleep(idle_rounds);
      }
    }
    __syncthreads();
    if (s_exit) break;
  }
  if (t == 0) {
    const uint32_t par = a.gen & 1u;
    const uint32_t prev = __hip_atomic_fetch_add(&a.dctl->wg_exited[par], 1u,
                                                 __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev + 1 == a.grid) {
      st_dev(&a.dctl->wg_exited[par], 0u);
      st_sys_rel(&a.hctl->exited[par], a.gen);
    }
  }
}

// The full variant asks for two waves per SIMD (at most 256 registers,
// accumulation registers included): two workgroups per compute unit, which
// suits matrix tiles (64-deep bf16 slices, no register spills in the slice
// loops).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
drain_kernel_full(KArgs) {
  drain_body<true>(kargs());
}

// The same at three waves per SIMD (at most 168 registers) with 32-deep bf16
// slices (45 KB of LDS): three workgroups per compute unit.  The matrix tiles
// spill registers and run slower, escape-time tiles mixed with them run
// faster (more waves to dual-issue from); a system picks one of the two.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
drain_kernel_full3(KArgs) {
  drain_body<true, 32>(kargs());
}

// The full variant for systems that use 128 x 256 bf16 tiles (two
// workgroups per compute unit); its square matrix tiles are calls.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
drain_kernel_wide(KArgs) {
  drain_body<true, kBf16SliceK, true>(kargs());
}

// The light variant asks for five waves per SIMD (at most 96 registers).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5)))
drain_kernel_light(KArgs) {
  drain_body<false>(kargs());
}

// ---- host-side launch wrappers ------------------------------------------

hipError_t launch_plain(const KArgs& a, const Desc& d, uint32_t ntiles, hipStream_t s) {
  if (d.behavior == CAF_BHV_GEMM)
    hipLaunchKernelGGL(plain_kernel<true>, dim3(ntiles), dim3(kThreads), 0, s, a, d, ntiles);
  else
    hipLaunchKernelGGL(plain_kernel<false>, dim3(ntiles), dim3(kThreads), 0, s, a, d, ntiles);
  return hipGetLastError();
}

const void* plain_kernel_fn(bool full) {
  return full ? reinterpret_cast<const void*>(&plain_kernel<true>)
              : reinterpret_cast<const void*>(&plain_kernel<false>);
}

hipError_t launch_drain(const KArgs& a, hipStream_t s) {
  if (a.full && a.wide)
    hipLaunchKernelGGL(drain_kernel_wide, dim3(a.grid), dim3(kThreads), 0, s, a);
  else if (a.full && a.full_wgs == 3)
    hipLaunchKernelGGL(drain_kernel_full3, dim3(a.grid), dim3(kThreads), 0, s, a);
  else if (a.full) hipLaunchKernelGGL(drain_kernel_full, dim3(a.grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL(drain_kernel_light, dim3(a.grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t drain_occupancy(bool full, uint32_t full_wgs, bool wide, int* blocks_per_cu) {
  if (full && wide)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, drain_kernel_wide,
                                                        kThreads, 0);
  if (full && full_wgs == 3)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, drain_kernel_full3,
                                                        kThreads, 0);
  if (full)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, drain_kernel_full,
                                                        kThreads, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, drain_kernel_light,
                                                      kThreads, 0);
}

}  // namespace cafgpu
