// Internal layouts of the compute-actor library: the mailbox entry
// (descriptor), the completion record, the control blocks shared between
// the host runtime and the drain kernel, and the work-tile geometry.  Used
// by the host runtime and the device code of this library only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/caf_gpu.h"

namespace cafgpu {

constexpr uint32_t kMaxActors = 1024;
constexpr uint32_t kAliveWords = kMaxActors / 32;
constexpr uint32_t kThreads = 256;  // one workgroup = 4 wave64s
constexpr uint32_t kInlineBytes = 16;
constexpr uint32_t kMaxHops = 2;
constexpr uint32_t kMaxBatch = 1024;
constexpr uint32_t kSlotBits = 20;  // request id = (sequence << kSlotBits) | slot
constexpr uint32_t kMaxSlots = 1u << kSlotBits;
constexpr uint32_t kTanhTile = 4096;   // elements per tanh work tile
constexpr uint32_t kRowsumTile = 16;   // rows per row-sum work tile
constexpr uint32_t kMandelBlockW = 16; // a wave's pixel block: 4 rows x 16 columns
constexpr uint32_t kMandelBlockH = 4;
// Entries of the device tile map (global tile index -> slot); a power of two
// so the ring position is a mask.
constexpr uint32_t kTileMapCap = 1u << 22;
static_assert((kTileMapCap & (kTileMapCap - 1)) == 0, "tile map size is a power of two");

enum DescFlags : uint16_t {
  DF_FP64 = 1,       // Mandelbrot in double (else float)
  DF_BF16 = 2,       // GEMM inputs are bfloat16 (else float)
  DF_INLINE_IN = 4,  // echo input travels in the parameter block
  DF_INLINE_OUT = 8, // reply (<= 16 B) travels in the completion record
  DF_SEND = 16,      // no reply wanted; the completion only recycles the slot
  DF_NO_COMPLETE = 32, // plain mode, non-final pipeline stage: no completion record
  DF_RGBA = 64        // Mandelbrot colour reply: uint32 palette[min(count, numel - 1)],
                      // palette at in0, its length in numel
};

// One message: a 128-byte mailbox entry.
struct alignas(16) Desc {
  uint64_t req_id;     // 0
  uint32_t slot;       // 8: index of the request's device slot
  uint32_t actor;      // 12: actor index
  uint16_t behavior;   // 16
  uint16_t flags;      // 18
  uint32_t seq;        // 20: per-actor sequence number (stateful ordering)
  uint64_t in0;        // 24: device pointers of the inputs ...
  uint64_t in1;        // 32
  uint64_t out;        // 40: ... and of the reply (the kernel's last parameter)
  uint32_t hop_actor[kMaxHops];  // 48: forwarding chain, actor index + 1 (0 = none)
  uint64_t hop_out[kMaxHops];    // 56: reply buffers of the hops
  uint32_t tcfg;       // 72: work-tile size (GEMM tile edge / Mandelbrot px per tile)
  uint32_t numel;      // 76: echo element count
  union {              // 80: parameter block, 48 bytes
    struct {
      double re_min, im_min, step_re, step_im;
      uint32_t width, row0, rows, max_iter;
    } m64;
    struct {
      float re_min, im_min, step_re, step_im;
      uint32_t pad[4];
      uint32_t width, row0, rows, max_iter;
    } m32;
    struct { uint32_t n, unit; } g;  // unit: output tiles per work unit (0: 1)
    struct { uint32_t rows, cols; } s;
    struct { uint64_t x; } h;
    uint8_t raw[48];
  } p;
};
static_assert(sizeof(Desc) == 128, "descriptor is one 128-byte mailbox entry");

// One reply notification, written by the device into host memory.
struct alignas(32) Comp {
  uint64_t req_id;
  int32_t status;
  uint32_t lap;  // written last (release): position / capacity + 1
  uint8_t data[kInlineBytes];
};
static_assert(sizeof(Comp) == 32, "completion record is 32 bytes");

// Host-resident (pinned, coherent) control block.
struct alignas(64) HostCtl {
  uint64_t tail;      // mailbox entries published by the host
  uint8_t pad0[56];
  uint64_t drained;   // mailbox entries copied to the device (device writes)
  uint8_t pad1[56];
  uint32_t stop;         // host asks the drain kernel to exit
  uint32_t exited[2];    // by launch parity: generation whose workgroups all exited
  uint32_t retiring[2];  // by launch parity: generation that began to retire
  uint8_t pad2[44];
  uint32_t alive[kAliveWords];  // bit per actor
};

// Device-resident control block (agent-scope atomics only).  The hot
// counters sit on separate 128-byte lines (the L2 line size).
struct alignas(128) DevCtl {
  uint64_t tiles_claimed;  // reservation cursor (fetch_add)
  uint8_t p0[120];
  uint64_t tiles_pub;      // work tiles published (claimable below this)
  uint8_t p1[120];
  uint64_t tiles_done;     // tiles finished (flow control of the tile map)
  uint8_t p2[120];
  uint32_t drain_lock;
  uint8_t p3[124];
  uint64_t comp_tail;      // completion positions handed out
  uint8_t p4[120];
  uint64_t drained;        // mailbox entries drained
  uint32_t stop_seen;      // a drainer saw the host's stop flag
  uint32_t wg_exited[2];   // by launch parity: workgroups that left
  uint32_t retiring[2];    // by launch parity: generation that began to retire
  uint32_t backlog;        // the last drain pass left entries in the mailbox
  uint8_t p5[96];
};
static_assert(sizeof(DevCtl) == 6 * 128, "hot counters on separate 128-byte lines");

constexpr uint32_t kNopTile = 0xFFFFFFFFu;  // tile-map entry of a filler tile

struct alignas(16) DevSlot {
  Desc d;              // the message currently held by this slot
  uint64_t tile_base;  // first global tile index of the message
  uint32_t ntiles;
  uint32_t pad;
  uint8_t inline_out[kInlineBytes];
};

struct alignas(16) SlotState {
  uint32_t done;      // tiles finished of the current stage
  uint32_t decision;  // plain mode: 0 undecided, 1 run, 2 actor quit
  int32_t status;     // reply status carried along a pipeline
  uint32_t pad;
};

struct alignas(16) DevActor {
  uint64_t state;     // hash-chain state (device-resident actor state)
  uint32_t seq_done;  // messages of this actor handled so far
  uint32_t pad;
};

// Everything a kernel needs, passed by value.
struct KArgs {
  HostCtl* hctl;
  Desc* hring;
  Comp* comp;
  DevCtl* dctl;
  DevSlot* slots;
  SlotState* sstate;
  uint32_t* tile2slot;
  DevActor* actors;
  uint32_t cap, ccap, max_batch;
  uint64_t idle_ticks;    // persistent: exit after this many wall-clock ticks idle
  uint64_t wait_ticks;    // bound of any device-side wait
  uint32_t gen;           // launch generation
  uint32_t exit_on_empty; // batched mode
  uint32_t grouping;
  uint32_t grid;
  uint32_t full;          // drain launch variant: 1 = every behaviour, 0 = all but GEMM
  uint32_t full_wgs;      // workgroups per compute unit of the full variant (2 or 3)
  uint32_t wide;          // full launches use the variant with 128 x 256 bf16 tiles
};

// ---- work-tile geometry (host and device agree on it) -------------------

// A wave iterates a group of blocks at once, one pixel of each per lane:
// 2 block rows x 2 block columns (8 x 32 pixels) in float, 2 x 1 (8 x 16) in
// double.  Blocks are numbered group by group, groups row-major; the count
// includes the blocks of the partial groups at the right and bottom edges.
constexpr uint32_t kMandelGroupRows = 2;
__host__ __device__ constexpr uint32_t mandel_group_cols(bool fp64) { return fp64 ? 1u : 2u; }
__host__ __device__ inline uint32_t mandel_blocks(uint32_t width, uint32_t rows, bool fp64) {
  const uint32_t gc = mandel_group_cols(fp64);
  const uint32_t bw = (width + kMandelBlockW - 1) / kMandelBlockW;
  const uint32_t bh = (rows + kMandelBlockH - 1) / kMandelBlockH;
  return ((bw + gc - 1) / gc) * ((bh + kMandelGroupRows - 1) / kMandelGroupRows) * gc *
         kMandelGroupRows;
}

// A product's output tiles (tcfg x tcfg blocks of C) and the work units
// they are claimed and completed in: `unit` consecutive tiles in row-major
// tile order.  A unit that covers a whole product completes it without the
// shared tile count and the release before it; units of several tiles
// therefore suit products whose tiles are short next to that release.
// tcfg 64 or 128: square tiles of that edge; 256: 128 x 256 tiles (bf16).
__host__ __device__ inline uint32_t gemm_tiles(const Desc& d) {
  if (d.tcfg == 256) return ((d.p.g.n + 127) / 128) * ((d.p.g.n + 255) / 256);
  const uint32_t t = (d.p.g.n + d.tcfg - 1) / d.tcfg;
  return t * t;
}
__host__ __device__ inline uint32_t gemm_unit(const Desc& d) { return d.p.g.unit ? d.p.g.unit : 1u; }
// bf16 products: four tiles per unit.  A 128 x 128 bf16 tile is short next
// to the agent-scope release (an L2 writeback) that a partial run needs, so
// a product of up to four tiles completes whole; fp32 tiles are long
// enough that single tiles end a batch more evenly.
constexpr uint32_t kGemmUnitBf16 = 4;

// Claimable work units of a message (the drain's "tiles").
__host__ __device__ inline uint32_t desc_ntiles(const Desc& d) {
  switch (d.behavior) {
    case CAF_BHV_MANDELBROT: {
      uint32_t w = d.p.m64.width, r = d.p.m64.rows;  // same offsets in m32
      uint32_t bpt = d.tcfg / 64;
      uint32_t nb = mandel_blocks(w, r, (d.flags & DF_FP64) != 0);
      return nb == 0 ? 1u : (nb + bpt - 1) / bpt;  // an empty tile still replies
    }
    case CAF_BHV_GEMM: {
      const uint32_t u = gemm_unit(d);
      return (gemm_tiles(d) + u - 1) / u;
    }
    case CAF_BHV_TANH: {
      uint64_t ne = (uint64_t)d.p.s.rows * d.p.s.cols;
      return (uint32_t)((ne + kTanhTile - 1) / kTanhTile);
    }
    case CAF_BHV_ROWSUM:
      return (d.p.s.rows + kRowsumTile - 1) / kRowsumTile;
    default:
      return 1;
  }
}

// Completion notifications for one native driver: the poller thread pushes
// the tag of each resolved tagged future, the driver pops (single producer,
// single consumer).
struct DriveQ {
  uint32_t* buf = nullptr;
  uint64_t mask = 0;
  alignas(64) uint64_t head = 0;  // consumer
  alignas(64) uint64_t tail = 0;  // producer
};

// The CPU actors of the CPU+GPU split (offload.cpp): a worker pool owned by
// the system, created on first use and destroyed at shutdown.
struct CpuPool;
void cpu_pool_destroy(CpuPool* p);
CpuPool*& cpu_pool_of(caf_gpu_system* s);
std::mutex& offload_mu_of(caf_gpu_system* s);  // one split at a time per system
int device_of(const caf_gpu_system* s);
// The fixed staging array of caf_offload_mandel_noalloc and the bound on its
// request table (public limits, caf_gpu.h).
constexpr uint64_t kOffloadStageBytes = CAF_OFFLOAD_NOALLOC_STAGE_BYTES;
constexpr uint32_t kOffloadNoallocMaxTiles = CAF_OFFLOAD_NOALLOC_MAX_ROWS / 64;
// Looks up the address of `device`'s copy of that array (once per device;
// the device must be current).  CAF_OK or CAF_E_DEVICE.
int offload_stage_setup(int device);

}  // namespace cafgpu

// Request entry used by the native driver: like caf_gpu_request, and the
// poller pushes `tag` into `q` when the future resolves.  try_only: never
// wait for admission; a message that does not fit yet (mailbox or arena
// full, but it would fit an empty arena) returns kTryLater and is not
// counted as refused.
constexpr int kTryLater = -100;
int cafgpu_request_tagged(caf_gpu_system* sys, caf_actor dst, uint32_t sender, const void* args,
                          uint64_t args_bytes, const caf_buf* in, uint32_t n_in,
                          const caf_buf* out_or_null, caf_actor forward_to, caf_future** fut,
                          cafgpu::DriveQ* q, uint32_t tag, bool try_only = false);
bool cafgpu_blocking(const caf_gpu_system* sys);
int64_t cafgpu_future_issue_ns(const caf_future* f);
int64_t cafgpu_future_done_ns(const caf_future* f);
