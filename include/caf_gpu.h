/*
 * caf_gpu.h -- the compute actor on one MI355X (gfx950), as a C ABI.
 *
 * A compute actor is an actor whose message handler is a data-parallel GPU
 * kernel (paper Sec. 4.6, "Transparent Integration of GPGPU Hardware
 * Components": an OpenCL kernel is wrapped as an actor that receives its
 * input arrays in a message, runs the kernel, and replies with the output
 * array, the kernel's last parameter; element counts are fixed when the
 * actor is spawned).  The calls below follow the paper's actor semantics:
 *
 *   caf_gpu_spawn    -- spawn_cl: create an actor bound to one behaviour
 *                       (kernel) and signature (Sec. 4.6, Sec. 4.5 typed
 *                       interfaces, checked here at run time).
 *   caf_gpu_send     -- asynchronous send, no reply (Sec. 5).
 *   caf_gpu_request  -- sync_send(...).then(...): the message gets a unique
 *                       id and exactly one reply, delivered through a
 *                       future; a dead receiver yields an error reply, and
 *                       the waiter may give up after a timeout (Sec. 5).
 *   caf_gpu_quit     -- the actor is done (Sec. 6 state machine); requests
 *                       it has not started get an error reply.
 *
 * Messages have call-by-value semantics (Sec. 4.4, copy-on-write): the
 * actor never writes its inputs, and each reply is a fresh buffer.
 *
 * Memory and streams: the caller hands in one device allocation (the
 * "arena", e.g. a PyTorch tensor) that bounds all device memory the library
 * uses for replies and staged inputs -- the HBM budget that admission
 * control enforces -- plus optional hipStream_t handles.  No PyTorch or C++
 * type crosses this interface.
 *
 * Status codes: calls return CAF_OK (0) or a negative CAF_E_* code; no C++
 * exception crosses the interface.  Errors that arise after a request was
 * accepted arrive as the reply status of its future.
 *
 * Threading: every call is thread-safe.  One host poller thread per system
 * resolves futures.
 */
#ifndef CAF_GPU_H
#define CAF_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CAF_OK = 0,
  CAF_E_INVALID = -1,  /* bad argument; dtype, shape or arity not in the actor's signature */
  CAF_E_NO_ACTOR = -2, /* no such actor, or it has quit */
  CAF_E_OVERLOAD = -3, /* non-blocking admission: HBM budget or mailbox full */
  CAF_E_TIMEOUT = -4,  /* the waiter gave up (the late reply is discarded) */
  CAF_E_DEVICE = -5,   /* HIP error, or a device-side wait ran out */
  CAF_E_QUIT = -6,     /* the actor quit before handling the message */
  CAF_E_FAULT = -7     /* the handler reported failure */
};

typedef enum {
  CAF_I32 = 0,
  CAF_U16 = 1,
  CAF_F32 = 2,
  CAF_F64 = 3,
  CAF_BF16 = 4, /* bfloat16 bit patterns, uint16 storage */
  CAF_U64 = 5,
  CAF_U32 = 6   /* colour-mapped Mandelbrot replies: one uint32 per pixel */
} caf_dtype;

/* Behaviours a compute actor can be bound to. */
typedef enum {
  CAF_BHV_NOOP = 0,       /* echo: reply = the int32 input (ping-pong) */
  CAF_BHV_MANDELBROT = 1, /* escape-time counts of a viewport tile -> uint16 */
  CAF_BHV_GEMM = 2,       /* C = A * B, square n x n, row-major, fp32 accumulate */
  CAF_BHV_TANH = 3,       /* elementwise tanh, f32 */
  CAF_BHV_ROWSUM = 4,     /* row sums of a rows x cols f32 matrix */
  CAF_BHV_HASHCHAIN = 5,  /* stateful: s = (s * 1000003) ^ x, reply s (u64) */
  CAF_BHV_FAULT = 6       /* always replies CAF_E_FAULT (tests error paths) */
} caf_behavior;

/* How messages reach the device. */
typedef enum {
  /* One kernel launch per message on the system stream (the baseline). */
  CAF_MODE_PLAIN = 0,
  /* Messages go through the mailbox ring; a drain kernel is launched when
   * work is waiting and exits when the ring is empty, so one launch serves
   * every message that arrived meanwhile. */
  CAF_MODE_BATCHED = 1,
  /* Messages go through the mailbox ring; a resident (persistent) drain
   * kernel polls it and exits only after idle_exit_us without work or at
   * shutdown; the library relaunches it when new work arrives. */
  CAF_MODE_PERSISTENT = 2,
  /* One launch per message like CAF_MODE_PLAIN, but each message's launches
   * (every stage of a pipeline) are replayed from an instantiated hipGraph,
   * one per stage shape (kernel variant and tile count of each stage); the
   * message's arguments are written into the graph's kernel nodes before
   * each replay.  At most 64 shapes are kept; further shapes launch
   * directly. */
  CAF_MODE_PLAIN_GRAPH = 3
} caf_mode;

/* Order in which a drained batch's work is laid out for the workgroups. */
typedef enum {
  CAF_GROUP_FIFO = 0, /* mailbox order */
  CAF_GROUP_LPT = 1,  /* grouped by behaviour, largest GEMMs first (stable) */
  CAF_GROUP_KIND = 2  /* grouped by behaviour, mailbox order within a group (stable) */
} caf_grouping;

typedef uint64_t caf_actor; /* actor address (Sec. 4.5 actor_addr); 0 is never valid */

/* A typed message buffer.  on_device = 1: data is device memory (HBM);
 * on_device = 0: host memory, which the library stages into the arena
 * before the actor sees it. */
typedef struct {
  void* data;
  uint64_t numel;
  int32_t dtype; /* caf_dtype */
  uint32_t on_device;
} caf_buf;

typedef struct caf_future caf_future;
typedef struct caf_gpu_system caf_gpu_system;

typedef struct {
  int32_t device;        /* HIP device ordinal */
  int32_t mode;          /* caf_mode */
  void* stream;          /* hipStream_t for plain launches and copies; NULL = own stream */
  void* drain_stream;    /* hipStream_t for the drain kernel; NULL = own stream */
  void* arena;           /* device memory for replies and staged inputs (the HBM budget) */
  uint64_t arena_bytes;
  uint32_t ring_slots;   /* max outstanding messages (mailbox capacity); 0 = 4096 */
  uint32_t max_batch;    /* messages drained per pass (the paper's max_msgs, Sec. 6); 0 = 1024 */
  uint32_t grid;         /* drain-kernel workgroups; 0 = chosen from occupancy */
  uint32_t blocking;     /* 1: requests wait for budget/mailbox space; 0: CAF_E_OVERLOAD */
  uint32_t idle_exit_us; /* drain kernel exits after this long without work;
                            0 = 200000 (persistent), 50 (batched) */
  int32_t grouping;      /* caf_grouping */
  uint32_t mandel_tile_px; /* pixels per Mandelbrot work tile (multiple of 256);
                              0 = 512 (plain), 1024 (batched / persistent) */
  uint32_t gemm_tile;      /* GEMM output tile edge (64 or 128) for every n, or 256 for
                              128 x 256 bf16 tiles; 0 = per class.  A 256 here or in
                              a class (ring modes, full_wgs_per_cu 2) gives them to
                              every bf16 product with n % 32 == 0 and 16-byte
                              aligned inputs; the others get 128 or their class's
                              edge */
  uint32_t gemm_tile_class[4]; /* the same choice for n <= 64, <= 128, <= 256, > 256;
                                  0 = default (64 up to n = 128, else 128) */
  uint32_t full_wgs_per_cu; /* drain workgroups per compute unit while a GEMM actor
                               exists: 0 or 2 = two (64-deep bf16 slices; suits
                               matrix-heavy loads), 3 = three (32-deep bf16
                               slices; more waves for escape-time tiles mixed
                               with products, slower matrix tiles) */
} caf_gpu_config;

/* Parameter blocks (the non-buffer part of a message), one per behaviour. */
typedef struct {
  double re_min, im_min;   /* lower-left corner of the whole image */
  double step_re, step_im; /* pixel pitch; pixel (x, y) samples re_min + x*step_re + i*(im_min + (row0+y)*step_im) */
  uint32_t width, height;  /* whole image size; width 1 .. 2^20 */
  uint32_t row0, rows;     /* this tile: global rows [row0, row0 + rows), rows <= 2^20,
                              rows * width <= 2^32 (else CAF_E_INVALID) */
  uint32_t max_iter;       /* 1 .. 65535 */
  int32_t fp;              /* CAF_F32 (viewport doubles rounded to float once) or CAF_F64 */
} caf_mandel_args;

typedef struct {
  uint32_t n;       /* square size */
  int32_t in_dtype; /* CAF_F32 or CAF_BF16; inputs A, B are n*n of it, reply is n*n f32 */
} caf_gemm_args;

typedef struct {
  uint32_t rows, cols; /* tanh: rows*cols f32 -> f32; rowsum: -> rows f32 */
} caf_shape_args;

typedef struct {
  uint64_t x; /* hash-chain input */
} caf_hash_args;

typedef struct {
  uint32_t n;           /* GEMM n, or tanh/rowsum rows (= cols); 0 = any size */
  uint32_t reserved;
  caf_actor forward_to; /* 0 = reply to the requester; else every reply becomes a request to it */
  /* Mandelbrot only: a data transformation fused into the handler (the
   * post-processing step spawn_cl accepts beside the kernel, Sec. 4.6).
   * With palette_len > 0 every reply is a colour image, CAF_U32
   * [rows][width], pixel = palette[min(count, palette_len - 1)]: the count
   * itself is never returned.  palette: device memory, palette_len
   * (1 .. 65536) entries, caller-owned, unchanged while the actor may still
   * handle a message.  Both 0: replies are the uint16 counts. */
  const uint32_t* palette;
  uint32_t palette_len;
  uint32_t reserved2;
} caf_spawn_args;

/* Creates a system on cfg->device.  The arena must stay allocated until
 * caf_gpu_shutdown.  Returns CAF_E_INVALID for a NULL/undersized arena or
 * bad sizes, CAF_E_DEVICE on a HIP failure. */
int caf_gpu_init(const caf_gpu_config* cfg, caf_gpu_system** out);

/* spawn_cl analog (Sec. 4.6): creates an actor bound to behavior; args may
 * be NULL.  The actor starts waiting for messages.  CAF_E_INVALID for an
 * unknown behaviour or forward target, or a palette that is not a
 * Mandelbrot actor's or not 1 .. 65536 entries at a non-NULL address;
 * CAF_E_OVERLOAD past 1024 actors. */
int caf_gpu_spawn(caf_gpu_system* sys, int32_t behavior, const caf_spawn_args* args,
                  caf_actor* out);

/* Asynchronous send (no reply).  args/args_bytes: the behaviour's parameter
 * block (copied).  in[0..n_in): input buffers; they must stay valid and
 * unmodified until the actor has handled the message (use a request when
 * the caller needs to know when).  Returns CAF_OK once enqueued in FIFO
 * order for (sender, actor); CAF_E_INVALID on a signature mismatch,
 * CAF_E_NO_ACTOR for a dead actor, CAF_E_OVERLOAD when full and
 * non-blocking. */
int caf_gpu_send(caf_gpu_system* sys, caf_actor dst, uint32_t sender, const void* args,
                 uint64_t args_bytes, const caf_buf* in, uint32_t n_in);

/* Request (sync_send): like caf_gpu_send, and *fut receives a future that
 * is resolved exactly once with the reply or an error.  out_or_null: a
 * caller-owned device buffer of the reply's dtype and size to write the
 * reply into; NULL = the library allocates it from the arena (owned by the
 * future until caf_future_release).  forward_to: 0, or an actor that
 * receives the reply as its input instead of the caller (and may forward
 * again per its spawn args); the last actor's reply resolves the future.
 * At most two forwarding hops. */
int caf_gpu_request(caf_gpu_system* sys, caf_actor dst, uint32_t sender, const void* args,
                    uint64_t args_bytes, const caf_buf* in, uint32_t n_in,
                    const caf_buf* out_or_null, caf_actor forward_to, caf_future** fut);

/* Waits up to timeout_ns (< 0: forever).  On resolution returns CAF_OK and
 * fills *result (the reply buffer: device memory, or host memory for
 * replies of at most 16 bytes, see on_device) and *reply_status (CAF_OK or
 * an error).  Returns CAF_E_TIMEOUT if the time ran out: the future is then
 * resolved with CAF_E_TIMEOUT and the late reply is discarded. */
int caf_future_wait(caf_future* fut, int64_t timeout_ns, caf_buf* result, int32_t* reply_status);

/* Non-blocking: 1 resolved (result/status filled), 0 pending, <0 error. */
int caf_future_poll(caf_future* fut, caf_buf* result, int32_t* reply_status);

/* The request id (unique per system). */
uint64_t caf_future_id(const caf_future* fut);

/* Gives the future and its arena reply buffer back (after a late reply
 * arrives, if it is still in flight). */
void caf_future_release(caf_future* fut);

/* The actor quits: requests it has not started are answered CAF_E_QUIT,
 * later messages are refused with CAF_E_NO_ACTOR.  A message being handled
 * completes normally. */
int caf_gpu_quit(caf_gpu_system* sys, caf_actor actor, uint32_t exit_reason);

/* become (Sec. 5.3, function-based actors; Sec. 5.4, class-based actors):
 * the actor's behaviour, signature and spawn arguments change for every
 * message submitted after this call; messages submitted before it are still
 * handled by the old behaviour (each carries its behaviour through the
 * mailbox), so the swap takes effect in mailbox order.  This is the
 * dynamically typed actor's become: the new behaviour may have another
 * signature (a statically typed actor would have to keep its interface).
 * The actor's device-resident state and the order in which its stateful
 * messages update it carry over.  CAF_E_NO_ACTOR for an unknown or quit
 * actor; CAF_E_INVALID for an unknown behaviour, forward target or palette
 * (as for caf_gpu_spawn). */
int caf_gpu_become(caf_gpu_system* sys, caf_actor actor, int32_t behavior,
                   const caf_spawn_args* args);

/* Holds the drain back (hold != 0) or lets it go (hold = 0); ring forms
 * only (CAF_E_INVALID for the plain forms, which launch at submit time).
 * While held, no drain kernel is launched: accepted messages wait in the
 * mailbox, up to ring_slots of them (beyond that requests wait or are
 * refused, as when the mailbox is full).  Letting go launches one drain for
 * everything that waited, which takes it in batches of max_batch -- the
 * caller sets a batch boundary, the way the scheduler's max_msgs bounds
 * what one actor run takes from its mailbox (Sec. 6).  A drain kernel that
 * is already running keeps draining; hold affects the next launch.
 * caf_gpu_drain waits for held messages (and times out while held). */
int caf_gpu_hold(caf_gpu_system* sys, int32_t hold);

/* Blocks until every accepted message is handled (all replies delivered). */
int caf_gpu_drain(caf_gpu_system* sys, int64_t timeout_ns);

/* Stops the drain kernel and the poller, answers anything left with
 * CAF_E_QUIT, frees library memory (not the caller's arena). */
int caf_gpu_shutdown(caf_gpu_system* sys);

const char* caf_gpu_strerror(int status);

/* Counters for tests and benchmarks. */
typedef struct {
  uint64_t requests, sends, completions;
  uint64_t launches;       /* plain-mode kernel launches */
  uint64_t drain_launches; /* drain-kernel launches (batched / persistent) */
  uint64_t duplicate_completions; /* completions for an unknown or reused id (must stay 0) */
  uint64_t swallowed;             /* late replies after a timeout */
  uint64_t arena_in_use, arena_peak;
  uint64_t rejected;              /* CAF_E_OVERLOAD returns */
  uint64_t device_drained;        /* mailbox entries drained by the device */
  uint64_t outstanding;           /* accepted messages not yet completed */
} caf_gpu_stats;

int caf_gpu_get_stats(caf_gpu_system* sys, caf_gpu_stats* out);

/* Total device time (ms, HIP events on the drain stream) of the drain-kernel
 * launches since the previous call, and their number in *launches.  Waits
 * for the drain stream to be idle.  Negative for a NULL system. */
double caf_gpu_drain_kernel_ms(caf_gpu_system* sys, uint64_t* launches);

/* ---- load driver -------------------------------------------------------
 * Issues a message list from native code, so that host-side Python overhead
 * does not limit message rates.  Each message is a request; its reply is
 * released as soon as it arrives, unless out[i].data is given (the reply is
 * then written there).
 *   window > 0, arrival_ns NULL: closed loop with at most `window`
 *     requests outstanding (window 1 = ping-pong).
 *   arrival_ns given: open loop; message i is issued at arrival_ns[i] after
 *     the start (scheduled time), latency counts from the scheduled time.
 *   chain_hops > 0: host-mediated forwarding, for comparison with
 *     device-side forwarding: every message's reply is re-sent by the host
 *     to hop_actor[0], then hop_actor[1] (shape args rows = cols = n).
 * latency_ns[i] (optional) gets reply time - issue/scheduled time;
 * status[i] (optional) the reply status.  Admission: the driver never waits
 * inside a request.  With a blocking system a request that does not fit
 * yet (mailbox or arena full) waits at the head of the driver's queue, in
 * order, and is retried as replies are harvested and released; with a
 * non-blocking system it is refused (status CAF_E_OVERLOAD, not counted as
 * an error).  Returns CAF_OK or the first other call-time error. */
typedef struct {
  caf_actor actor;
  uint32_t sender;
  uint32_t n_in;
  const void* args;
  uint64_t args_bytes;
  const caf_buf* in;
  caf_buf out; /* out.data == NULL: library-allocated, released on arrival */
  caf_actor forward_to;
} caf_msg;

int caf_gpu_drive(caf_gpu_system* sys, const caf_msg* msgs, uint64_t count, uint32_t window,
                  const int64_t* arrival_ns, uint32_t chain_hops, const caf_actor* hop_actor,
                  int64_t* latency_ns, int32_t* status, double* elapsed_s);

/* ---- CPU actors and the CPU+GPU split (Sec. 7.5) ------------------------
 * The paper's offload experiment computes one Mandelbrot image partly on
 * CPU actors and partly on a GPU compute actor and times the whole image as
 * the GPU's share grows.  These two calls are that experiment; the GPU path
 * never calls them.
 *
 * caf_cpu_mandel_rows: the CPU actors' kernel on the calling thread.  Global
 * rows [row_begin, row_end) of the image `a` describes (a->row0 and a->rows
 * are not used) are written to out_host, uint16 [row_end - row_begin][width]
 * row-major, caller-owned.  The counts equal the GPU behaviour's (same
 * recurrence, operation order and rounding).  Needs no device.  Returns
 * CAF_E_INVALID for a NULL pointer, a bad width, height, max_iter or fp, or
 * rows outside the image.
 *
 * caf_offload_mandel: the whole image `image` (row0 = 0, rows = height).
 * Rows [0, gpu_rows) go to `gpu_actor` (a Mandelbrot actor) as requests of
 * at most 64 rows whose replies are written into dev_stage (device memory,
 * at least gpu_rows * width uint16, caller-owned) and then copied to
 * out_host; at the same time rows [gpu_rows, height) are computed by
 * `cpu_threads` worker threads of the system (0 = one per hardware thread,
 * at most 1024; the pool is created on first use and kept until
 * caf_gpu_shutdown).
 * out_host: uint16 [height][width], caller-owned host memory.  times
 * (optional): wall time of the call, and when each share was complete in
 * host memory, from the start of the call.  Calls on one system run one at
 * a time.  Returns CAF_OK, CAF_E_INVALID for bad arguments, CAF_E_OVERLOAD
 * if the worker threads cannot be started, a call-time error of a request,
 * the first error reply, or CAF_E_DEVICE if the copy fails. */
typedef struct {
  int64_t total_ns;
  int64_t gpu_done_ns; /* the GPU share in out_host (0 if gpu_rows = 0) */
  int64_t cpu_done_ns; /* the CPU share in out_host (0 if gpu_rows = height) */
} caf_offload_times;

int caf_cpu_mandel_rows(const caf_mandel_args* a, uint32_t row_begin, uint32_t row_end,
                        uint16_t* out_host);
int caf_offload_mandel(caf_gpu_system* sys, caf_actor gpu_actor, const caf_mandel_args* image,
                       uint32_t gpu_rows, uint32_t cpu_threads, uint16_t* dev_stage,
                       uint16_t* out_host, caf_offload_times* times);

/* caf_offload_mandel_noalloc: for callers that cannot allocate (code that
 * must not call hipMalloc, harnesses that forbid it, tight serving loops).
 * The same split as caf_offload_mandel, with the same results, except that
 * the GPU share is staged in the library's own device array instead of a
 * caller's dev_stage: a fixed CAF_OFFLOAD_NOALLOC_STAGE_BYTES array per
 * device, held from the first caf_gpu_init on that device until the
 * process ends.  The call allocates no device or pinned host memory (no
 * hipMalloc, hipHostMalloc or hipFree, no arena bytes: the replies go to
 * the array), keeps its request table on the stack, and takes its requests'
 * futures from the system's pool (filled by caf_gpu_init).
 * Limits: gpu_rows * width * 2 <= CAF_OFFLOAD_NOALLOC_STAGE_BYTES and
 * gpu_rows <= CAF_OFFLOAD_NOALLOC_MAX_ROWS, else CAF_E_INVALID; a CPU share
 * (gpu_rows < height) needs the system's CPU actors to be running with
 * cpu_threads workers already (an earlier caf_offload_mandel call with the
 * same cpu_threads starts them), else CAF_E_INVALID, since starting threads
 * allocates.  Every call on one device shares that device's array and
 * leaves its GPU share there: calls on one system run one at a time, but
 * calls from two systems on the same device that overlap race on the
 * array.  Other errors as caf_offload_mandel; CAF_E_DEVICE if the array's
 * address could not be found. */
#define CAF_OFFLOAD_NOALLOC_STAGE_BYTES (16u << 20)
#define CAF_OFFLOAD_NOALLOC_MAX_ROWS 16384u
int caf_offload_mandel_noalloc(caf_gpu_system* sys, caf_actor gpu_actor,
                               const caf_mandel_args* image, uint32_t gpu_rows,
                               uint32_t cpu_threads, uint16_t* out_host,
                               caf_offload_times* times);

#ifdef __cplusplus
}
#endif
#endif /* CAF_GPU_H */
