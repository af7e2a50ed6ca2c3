/*
 * cafref -- the CPU oracle for the compute-actor hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the GPU path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product library never links, loads or calls it, and the two share
 * no source, header, table or helper.
 *
 * It implements, single threaded and in the order the paper states them:
 *   - an actor runtime: one FIFO mailbox per actor (a mailbox is a queue that
 *     only its owner reads and anyone may append to, Sec. 2 and Sec. 4.3),
 *     request/reply with a unique request id and exactly one reply
 *     (Sec. 5, the sync_send / then discussion), quit with error replies for
 *     pending requests (the error-handling remark in the same passage), and
 *     compute actors whose handler is a kernel whose last parameter is the
 *     output (Sec. 4.6, the OpenCL actor / spawn_cl passage);
 *   - scalar kernels: Mandelbrot escape time in float and double (the
 *     Mandelbrot workloads of Sec. 7.4 and Sec. 7.5; the paper gives no
 *     formula, so the textbook escape-time rule is used, see the readings
 *     list of the design notes), the dense product of two flat n x n matrices
 *     in double (Sec. 4.6, the matrix_multiply kernel prototype), tanh,
 *     row sums, echo and a non-commutative hash chain.
 *
 * Build: g++ -O2 -ffp-contract=off (no -ffast-math): every floating point
 * operation is rounded to its own type, in the order written.
 */
#ifndef CAFREF_H
#define CAFREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reply / call status codes.  Their values mean the same as the GPU
 * library's, so tests can compare statuses directly. */
enum {
  REF_OK = 0,
  REF_E_INVALID = -1,
  REF_E_NO_ACTOR = -2,
  REF_E_OVERLOAD = -3,
  REF_E_TIMEOUT = -4,
  REF_E_DEVICE = -5,
  REF_E_QUIT = -6,
  REF_E_FAULT = -7
};

/* Element types of message buffers. */
enum { REF_I32 = 0, REF_U16 = 1, REF_F32 = 2, REF_F64 = 3, REF_BF16 = 4, REF_U64 = 5 };

/* Behaviours (message handlers) a compute actor can be bound to. */
enum {
  REF_BHV_NOOP = 0,       /* echo: reply = the int32 input */
  REF_BHV_MANDELBROT = 1, /* escape-time counts of a viewport tile */
  REF_BHV_GEMM = 2,       /* C = A * B, n x n, flat row-major */
  REF_BHV_TANH = 3,       /* elementwise tanh */
  REF_BHV_ROWSUM = 4,     /* per-row sum of a rows x cols matrix */
  REF_BHV_HASHCHAIN = 5,  /* stateful: s = (s * 1000003) ^ x */
  REF_BHV_FAULT = 6       /* always replies with REF_E_FAULT */
};

/* ---- scalar kernels -------------------------------------------------- */

/* Escape-time counts of one tile of a viewport.  Pixel (x, y) of the tile
 * samples c = (re_min + x * step_re) + i (im_min + (row0 + y) * step_im)
 * (lower-left corner sampling, global row index), iterates z <- z^2 + c
 * from z = 0 while |z|^2 <= 4, and stores the number of iterations taken
 * before the first |z_n|^2 > 4, or max_iter.  out has rows * width uint16
 * entries, row-major.  The float variant rounds the four doubles to float
 * once, then computes every operation in float. */
void caf_ref_mandelbrot_f32(double re_min, double im_min, double step_re, double step_im,
                            uint32_t width, uint32_t row0, uint32_t rows, uint32_t max_iter,
                            uint16_t* out);
void caf_ref_mandelbrot_f64(double re_min, double im_min, double step_re, double step_im,
                            uint32_t width, uint32_t row0, uint32_t rows, uint32_t max_iter,
                            uint16_t* out);

/* C[i][j] = sum_k A[i][k] * B[k][j] in double, k ascending; A, B row-major
 * n x n.  The _bf16 variant takes bfloat16 bit patterns and widens them
 * exactly. */
void caf_ref_gemm_f32(uint32_t n, const float* A, const float* B, double* C);
void caf_ref_gemm_bf16(uint32_t n, const uint16_t* A, const uint16_t* B, double* C);
void caf_ref_tanh_f64(uint64_t count, const double* x, double* y);
void caf_ref_rowsum_f64(uint32_t rows, uint32_t cols, const double* x, double* y);
uint64_t caf_ref_hash_step(uint64_t s, uint64_t x);

/* ---- actor runtime ---------------------------------------------------- */

typedef struct ref_system ref_system;

typedef struct {
  const void* data;   /* host memory */
  uint64_t numel;
  int32_t dtype;      /* REF_* element type */
} ref_buf;

/* Parameter blocks, one per behaviour. */
typedef struct {
  double re_min, im_min, step_re, step_im;
  uint32_t width, height, row0, rows, max_iter;
  int32_t fp; /* REF_F32 or REF_F64 */
} ref_mandel_args;

typedef struct {
  uint32_t n;
  int32_t in_dtype; /* REF_F32 or REF_BF16 */
} ref_gemm_args;

typedef struct {
  uint32_t rows, cols;
} ref_shape_args;

/* Spawn arguments: the signature the actor accepts (checked on every
 * message) and, for pipeline stages, the actor each reply is forwarded to. */
typedef struct {
  uint32_t n;          /* GEMM n; tanh/rowsum rows (= cols); 0 = any */
  uint64_t forward_to; /* 0 = reply to the requester */
} ref_spawn_args;

ref_system* caf_ref_new(void);
void caf_ref_free(ref_system* sys);
int caf_ref_spawn(ref_system* sys, int32_t behavior, const ref_spawn_args* args, uint64_t* actor);
/* Fire-and-forget message (no reply). */
int caf_ref_send(ref_system* sys, uint64_t actor, uint32_t sender, const void* args,
                 uint64_t args_bytes, const ref_buf* in, uint32_t n_in);
/* Request: a unique id is returned in *req; exactly one reply will be set. */
int caf_ref_request(ref_system* sys, uint64_t actor, uint32_t sender, const void* args,
                    uint64_t args_bytes, const ref_buf* in, uint32_t n_in, uint64_t forward_to,
                    uint64_t* req);
/* Run every actor until all mailboxes are empty.  Returns messages handled. */
uint64_t caf_ref_run(ref_system* sys);
/* Quit: pending requests in the mailbox are answered with REF_E_QUIT,
 * pending sends are dropped, later messages are refused with REF_E_NO_ACTOR. */
int caf_ref_quit(ref_system* sys, uint64_t actor, uint32_t reason);
/* Reply of a request.  Returns 1 if resolved, 0 if pending, <0 if unknown.
 * Copies min(cap, bytes) reply bytes to out; *bytes gets the full size,
 * *dtype the element type, *resolutions how many times it was resolved. */
int caf_ref_reply(ref_system* sys, uint64_t req, int32_t* status, void* out, uint64_t cap,
                  uint64_t* bytes, int32_t* dtype, uint32_t* resolutions);
/* Times out a pending request (as a waiter that gives up would): it is
 * resolved with REF_E_TIMEOUT and a later reply is swallowed. */
int caf_ref_timeout(ref_system* sys, uint64_t req);
/* The order in which an actor dequeued messages: (sender, per-sender seq). */
uint64_t caf_ref_dequeue_log(ref_system* sys, uint64_t actor, uint32_t* senders, uint32_t* seqs,
                             uint64_t cap);
uint64_t caf_ref_actor_state(ref_system* sys, uint64_t actor);
/* become (Sec. 5.3, function-based actors; Sec. 5.4, class-based actors):
 * the actor's behaviour and signature change for every message enqueued
 * after this call (a dynamically typed actor's become); earlier ones still
 * meet the old behaviour (the change travels through the mailbox as a
 * control entry, in order).  The actor's state is kept.  REF_E_NO_ACTOR for an unknown or
 * quit actor, REF_E_INVALID for a bad behaviour or forward target. */
int caf_ref_become(ref_system* sys, uint64_t actor, int32_t behavior, const ref_spawn_args* args);

#ifdef __cplusplus
}
#endif
#endif
