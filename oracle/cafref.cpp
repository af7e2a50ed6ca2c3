// cafref -- CPU oracle for the compute-actor hot path.
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
// CPU-baseline leg of the benchmark, never by the product library.  Shares no
// code with the GPU path.  Built with -O2 -ffp-contract=off and no
// -ffast-math, so every floating point operation below is one IEEE
// round-to-nearest operation in the type written, in the order written.
//
// Parity status: every function here is pinned by the CPU test suite
// (closed-form orbits, symmetry, the parabolic-point asymptote, brute force
// against exact rational arithmetic and a library matrix product, runtime
// ordering and exactly-once properties); nothing is "parity unpinned".
#include "cafref.h"

#include <cmath>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <vector>

// ---------------------------------------------------------------------------
// Mandelbrot escape time.
//
// The paper offloads "the calculation of the Mandelbrot set" (Sec. 7.4, the
// Benchmarks Game program, and Sec. 7.5, the OpenCL-actor experiment over a
// 1920x1080 viewport) without stating the recurrence.  This is the textbook
// set definition -- c is in the set iff the orbit of 0 under z <- z^2 + c stays
// within |z| <= 2 -- read as an escape-time count:
//   z_0 = 0, z_{k+1} = z_k^2 + c,
//   count = the first k with |z_k|^2 > 4 (strict), or max_iter if none of
//           z_0 .. z_{max_iter-1} escapes.
// Op order per iteration: zr2 = zr*zr; zi2 = zi*zi; test zr2 + zi2 > 4;
// t = zr*zi; zi = (t + t) + ci; zr = (zr2 - zi2) + cr.
// Pixel (x, y) of a tile samples its lower-left corner with the *global* row
// index row0 + y:  cr = re_min + x*step_re;  ci = im_min + (row0+y)*step_im
// (multiply, then add, each rounded).
// ---------------------------------------------------------------------------
template <typename T>
static uint16_t escape_count(T cr, T ci, uint32_t max_iter) {
  T zr = 0, zi = 0;
  uint32_t n = 0;
  while (n < max_iter) {
    T zr2 = zr * zr;
    T zi2 = zi * zi;
    T mag = zr2 + zi2;
    if (mag > T(4)) break;
    T t = zr * zi;
    T tt = t + t;
    zi = tt + ci;
    T d = zr2 - zi2;
    zr = d + cr;
    n = n + 1;
  }
  return (uint16_t)n;
}

template <typename T>
static void mandelbrot_tile(T re_min, T im_min, T step_re, T step_im, uint32_t width,
                            uint32_t row0, uint32_t rows, uint32_t max_iter, uint16_t* out) {
  for (uint32_t y = 0; y < rows; ++y) {
    T gy = (T)(row0 + y);
    T ym = gy * step_im;
    T ci = im_min + ym;
    for (uint32_t x = 0; x < width; ++x) {
      T gx = (T)x;
      T xm = gx * step_re;
      T cr = re_min + xm;
      out[(uint64_t)y * width + x] = escape_count<T>(cr, ci, max_iter);
    }
  }
}

extern "C" void caf_ref_mandelbrot_f32(double re_min, double im_min, double step_re,
                                       double step_im, uint32_t width, uint32_t row0,
                                       uint32_t rows, uint32_t max_iter, uint16_t* out) {
  // Float messages: the four viewport doubles are rounded to float once.
  mandelbrot_tile<float>((float)re_min, (float)im_min, (float)step_re, (float)step_im, width,
                         row0, rows, max_iter, out);
}

extern "C" void caf_ref_mandelbrot_f64(double re_min, double im_min, double step_re,
                                       double step_im, uint32_t width, uint32_t row0,
                                       uint32_t rows, uint32_t max_iter, uint16_t* out) {
  mandelbrot_tile<double>(re_min, im_min, step_re, step_im, width, row0, rows, max_iter, out);
}

// ---------------------------------------------------------------------------
// Dense matrix product (Sec. 4.6: matrix_multiply takes two flat arrays and
// writes the product to its last parameter; matrices are stored in one
// dimension, read here as row-major).  Exact definition, in double, with the
// inner index ascending.
// ---------------------------------------------------------------------------
static double bf16_to_double(uint16_t h) {
  uint32_t bits = (uint32_t)h << 16;  // bfloat16 is the top half of a float
  float f;
  std::memcpy(&f, &bits, 4);
  return (double)f;
}

extern "C" void caf_ref_gemm_f32(uint32_t n, const float* A, const float* B, double* C) {
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (uint32_t k = 0; k < n; ++k)
        acc += (double)A[(uint64_t)i * n + k] * (double)B[(uint64_t)k * n + j];
      C[(uint64_t)i * n + j] = acc;
    }
}

extern "C" void caf_ref_gemm_bf16(uint32_t n, const uint16_t* A, const uint16_t* B, double* C) {
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (uint32_t k = 0; k < n; ++k)
        acc += bf16_to_double(A[(uint64_t)i * n + k]) * bf16_to_double(B[(uint64_t)k * n + j]);
      C[(uint64_t)i * n + j] = acc;
    }
}

extern "C" void caf_ref_tanh_f64(uint64_t count, const double* x, double* y) {
  for (uint64_t i = 0; i < count; ++i) y[i] = std::tanh(x[i]);
}

extern "C" void caf_ref_rowsum_f64(uint32_t rows, uint32_t cols, const double* x, double* y) {
  for (uint32_t r = 0; r < rows; ++r) {
    double acc = 0.0;
    for (uint32_t c = 0; c < cols; ++c) acc += x[(uint64_t)r * cols + c];
    y[r] = acc;
  }
}

// A non-commutative fold (arithmetic mod 2^64), so any reordering of the
// messages an actor handles changes its final state.
extern "C" uint64_t caf_ref_hash_step(uint64_t s, uint64_t x) {
  return (s * 1000003ull) ^ x;
}

// ---------------------------------------------------------------------------
// Actor runtime.
//
// Sec. 2 / Sec. 4.3: a mailbox is a FIFO that only its owner dequeues from
// and that anyone may enqueue to.  Sec. 5: a synchronous send gets a unique
// id and exactly one response (or an error / timeout).  Sec. 4.6: a compute
// actor's reply is the kernel's output buffer.  Sec. 6: an actor is waiting,
// ready, running or done; here run() visits actors round-robin and handles
// one message per visit until every mailbox is empty.
// ---------------------------------------------------------------------------
namespace {

struct Msg {
  uint64_t req;  // 0 for a plain send
  uint32_t sender;
  uint32_t seq;  // per (sender, actor) sequence number
  std::vector<uint8_t> args;
  std::vector<std::vector<uint8_t>> in;
  std::vector<int32_t> in_dtype;
  std::vector<uint64_t> in_numel;
  uint64_t forward_to;
  bool become = false;  // a control entry: switch the behaviour when dequeued
  int32_t become_behavior = 0;
  ref_spawn_args become_spawn{0, 0};
};

struct Actor {
  int32_t behavior;  // the behaviour the next dequeued message meets
  ref_spawn_args spawn;
  int32_t tail_behavior;  // ... and the one a message enqueued now will meet
  ref_spawn_args tail_spawn;
  bool alive;
  uint64_t state;  // hash-chain state
  std::deque<Msg> mailbox;
  std::unordered_map<uint32_t, uint32_t> next_seq;  // per sender
  std::vector<std::pair<uint32_t, uint32_t>> log;   // dequeue order
};

struct Reply {
  bool resolved = false;
  int32_t status = 0;
  int32_t dtype = 0;
  uint32_t resolutions = 0;
  std::vector<uint8_t> bytes;
};

size_t dtype_size(int32_t dt) {
  switch (dt) {
    case REF_I32: return 4;
    case REF_U16: return 2;
    case REF_F32: return 4;
    case REF_F64: return 8;
    case REF_BF16: return 2;
    case REF_U64: return 8;
  }
  return 0;
}

}  // namespace

struct ref_system {
  std::vector<Actor> actors;  // actor id = index + 1
  std::unordered_map<uint64_t, Reply> replies;
  uint64_t next_req = 1;
};

static Actor* find_actor(ref_system* s, uint64_t id) {
  if (id == 0 || id > s->actors.size()) return nullptr;
  return &s->actors[id - 1];
}

static void resolve(ref_system* s, uint64_t req, int32_t status, int32_t dtype,
                    std::vector<uint8_t>&& bytes) {
  if (req == 0) return;
  Reply& r = s->replies[req];
  r.resolutions += 1;
  if (r.resolved) return;  // a late reply after a timeout is swallowed
  r.resolved = true;
  r.status = status;
  r.dtype = dtype;
  r.bytes = std::move(bytes);
}

// Checks a message against the actor's signature (Sec. 4.5 typed
// interfaces, Sec. 4.6 element counts fixed at spawn).  Returns REF_OK or
// REF_E_INVALID.
static int check_signature(int32_t behavior, const ref_spawn_args& spawn, const void* args,
                           uint64_t args_bytes, const ref_buf* in, uint32_t n_in) {
  switch (behavior) {
    case REF_BHV_NOOP:
      if (n_in != 1 || in[0].dtype != REF_I32 || in[0].numel == 0) return REF_E_INVALID;
      return REF_OK;
    case REF_BHV_MANDELBROT: {
      if (n_in != 0 || args_bytes != sizeof(ref_mandel_args)) return REF_E_INVALID;
      const ref_mandel_args* m = (const ref_mandel_args*)args;
      if (m->max_iter < 1 || m->max_iter > 65535) return REF_E_INVALID;
      if (m->width == 0 || m->fp < REF_F32 || m->fp > REF_F64) return REF_E_INVALID;
      if ((uint64_t)m->row0 + m->rows > m->height) return REF_E_INVALID;
      return REF_OK;
    }
    case REF_BHV_GEMM: {
      if (args_bytes != sizeof(ref_gemm_args) || n_in != 2) return REF_E_INVALID;
      const ref_gemm_args* g = (const ref_gemm_args*)args;
      if (g->n == 0 || (g->in_dtype != REF_F32 && g->in_dtype != REF_BF16)) return REF_E_INVALID;
      if (spawn.n != 0 && spawn.n != g->n) return REF_E_INVALID;
      uint64_t nn = (uint64_t)g->n * g->n;
      for (uint32_t i = 0; i < 2; ++i)
        if (in[i].dtype != g->in_dtype || in[i].numel != nn) return REF_E_INVALID;
      return REF_OK;
    }
    case REF_BHV_TANH:
    case REF_BHV_ROWSUM: {
      if (args_bytes != sizeof(ref_shape_args) || n_in != 1) return REF_E_INVALID;
      const ref_shape_args* sh = (const ref_shape_args*)args;
      if (sh->rows == 0 || sh->cols == 0) return REF_E_INVALID;
      if (spawn.n != 0 && (spawn.n != sh->rows || spawn.n != sh->cols)) return REF_E_INVALID;
      if (in[0].dtype != REF_F32 && in[0].dtype != REF_F64) return REF_E_INVALID;
      if (in[0].numel != (uint64_t)sh->rows * sh->cols) return REF_E_INVALID;
      return REF_OK;
    }
    case REF_BHV_HASHCHAIN:
      if (n_in != 0 || args_bytes != 8) return REF_E_INVALID;
      return REF_OK;
    case REF_BHV_FAULT:
      return REF_OK;
  }
  return REF_E_INVALID;
}

extern "C" ref_system* caf_ref_new(void) { return new ref_system(); }
extern "C" void caf_ref_free(ref_system* sys) { delete sys; }

extern "C" int caf_ref_spawn(ref_system* sys, int32_t behavior, const ref_spawn_args* args,
                             uint64_t* actor) {
  if (behavior < REF_BHV_NOOP || behavior > REF_BHV_FAULT || actor == nullptr)
    return REF_E_INVALID;
  Actor a;
  a.behavior = behavior;
  a.spawn = args ? *args : ref_spawn_args{0, 0};
  a.tail_behavior = a.behavior;
  a.tail_spawn = a.spawn;
  a.alive = true;
  a.state = 0;
  sys->actors.push_back(std::move(a));
  *actor = sys->actors.size();
  return REF_OK;
}

static int enqueue(ref_system* sys, uint64_t actor, uint32_t sender, const void* args,
                   uint64_t args_bytes, const ref_buf* in, uint32_t n_in, uint64_t forward_to,
                   uint64_t req) {
  Actor* a = find_actor(sys, actor);
  if (a == nullptr || !a->alive) return REF_E_NO_ACTOR;
  int st = check_signature(a->tail_behavior, a->tail_spawn, args, args_bytes, in, n_in);
  if (st != REF_OK) return st;
  if (forward_to != 0) {
    Actor* f = find_actor(sys, forward_to);
    if (f == nullptr || !f->alive) return REF_E_NO_ACTOR;
  }
  Msg m;
  m.req = req;
  m.sender = sender;
  m.seq = a->next_seq[sender]++;
  m.args.assign((const uint8_t*)args, (const uint8_t*)args + args_bytes);
  for (uint32_t i = 0; i < n_in; ++i) {
    size_t nb = in[i].numel * dtype_size(in[i].dtype);
    // Call-by-value (Sec. 4.4): the message owns a copy of its inputs.
    m.in.emplace_back((const uint8_t*)in[i].data, (const uint8_t*)in[i].data + nb);
    m.in_dtype.push_back(in[i].dtype);
    m.in_numel.push_back(in[i].numel);
  }
  m.forward_to = forward_to;
  a->mailbox.push_back(std::move(m));
  return REF_OK;
}

extern "C" int caf_ref_send(ref_system* sys, uint64_t actor, uint32_t sender, const void* args,
                            uint64_t args_bytes, const ref_buf* in, uint32_t n_in) {
  return enqueue(sys, actor, sender, args, args_bytes, in, n_in, 0, 0);
}

extern "C" int caf_ref_request(ref_system* sys, uint64_t actor, uint32_t sender,
                               const void* args, uint64_t args_bytes, const ref_buf* in,
                               uint32_t n_in, uint64_t forward_to, uint64_t* req) {
  uint64_t id = sys->next_req;
  int st = enqueue(sys, actor, sender, args, args_bytes, in, n_in, forward_to, id);
  if (st != REF_OK) return st;
  sys->next_req += 1;
  sys->replies[id] = Reply();
  *req = id;
  return REF_OK;
}

static std::vector<double> widen(const std::vector<uint8_t>& raw, int32_t dtype, uint64_t n) {
  std::vector<double> v(n);
  if (dtype == REF_F64) {
    std::memcpy(v.data(), raw.data(), n * 8);
  } else {
    const float* f = (const float*)raw.data();
    for (uint64_t i = 0; i < n; ++i) v[i] = (double)f[i];
  }
  return v;
}

template <typename V>
static std::vector<uint8_t> as_bytes(const std::vector<V>& v) {
  std::vector<uint8_t> b(v.size() * sizeof(V));
  if (!b.empty()) std::memcpy(b.data(), v.data(), b.size());
  return b;
}

// Runs one message through the actor's behaviour.  Produces the reply (or
// forwards it, Sec. 5 "redistribute tasks" between actors).
static void handle(ref_system* sys, uint64_t actor_id, Msg& m) {
  Actor& a = sys->actors[actor_id - 1];
  if (m.become) {
    a.behavior = m.become_behavior;
    a.spawn = m.become_spawn;
    return;
  }
  a.log.emplace_back(m.sender, m.seq);
  int32_t status = REF_OK;
  int32_t dtype = REF_U16;
  std::vector<uint8_t> out;
  uint32_t out_rows = 0, out_cols = 0;
  switch (a.behavior) {
    case REF_BHV_NOOP:
      dtype = REF_I32;
      out = m.in[0];
      break;
    case REF_BHV_MANDELBROT: {
      ref_mandel_args g;
      std::memcpy(&g, m.args.data(), sizeof g);
      std::vector<uint16_t> px((uint64_t)g.rows * g.width);
      if (g.fp == REF_F32)
        caf_ref_mandelbrot_f32(g.re_min, g.im_min, g.step_re, g.step_im, g.width, g.row0, g.rows,
                               g.max_iter, px.data());
      else
        caf_ref_mandelbrot_f64(g.re_min, g.im_min, g.step_re, g.step_im, g.width, g.row0, g.rows,
                               g.max_iter, px.data());
      dtype = REF_U16;
      out = as_bytes(px);
      out_rows = g.rows;
      out_cols = g.width;
      break;
    }
    case REF_BHV_GEMM: {
      ref_gemm_args g;
      std::memcpy(&g, m.args.data(), sizeof g);
      std::vector<double> c((uint64_t)g.n * g.n);
      if (g.in_dtype == REF_F32)
        caf_ref_gemm_f32(g.n, (const float*)m.in[0].data(), (const float*)m.in[1].data(),
                         c.data());
      else
        caf_ref_gemm_bf16(g.n, (const uint16_t*)m.in[0].data(), (const uint16_t*)m.in[1].data(),
                          c.data());
      dtype = REF_F64;
      out = as_bytes(c);
      out_rows = out_cols = g.n;
      break;
    }
    case REF_BHV_TANH: {
      ref_shape_args sh;
      std::memcpy(&sh, m.args.data(), sizeof sh);
      std::vector<double> x = widen(m.in[0], m.in_dtype[0], m.in_numel[0]);
      std::vector<double> y(x.size());
      caf_ref_tanh_f64(x.size(), x.data(), y.data());
      dtype = REF_F64;
      out = as_bytes(y);
      out_rows = sh.rows;
      out_cols = sh.cols;
      break;
    }
    case REF_BHV_ROWSUM: {
      ref_shape_args sh;
      std::memcpy(&sh, m.args.data(), sizeof sh);
      std::vector<double> x = widen(m.in[0], m.in_dtype[0], m.in_numel[0]);
      std::vector<double> y(sh.rows);
      caf_ref_rowsum_f64(sh.rows, sh.cols, x.data(), y.data());
      dtype = REF_F64;
      out = as_bytes(y);
      out_rows = sh.rows;
      out_cols = 1;
      break;
    }
    case REF_BHV_HASHCHAIN: {
      uint64_t x;
      std::memcpy(&x, m.args.data(), 8);
      a.state = caf_ref_hash_step(a.state, x);
      dtype = REF_U64;
      out = as_bytes(std::vector<uint64_t>{a.state});
      break;
    }
    case REF_BHV_FAULT:
      status = REF_E_FAULT;
      break;
  }
  if (m.req == 0) return;  // a send: the result is discarded
  uint64_t next = m.forward_to != 0 ? m.forward_to : a.spawn.forward_to;
  if (status == REF_OK && next != 0) {
    // The reply becomes a request to the next actor, carrying the same id.
    Actor* f = find_actor(sys, next);
    if (f == nullptr || !f->alive) {
      resolve(sys, m.req, REF_E_QUIT, 0, {});
      return;
    }
    ref_shape_args sh{out_rows, out_cols};
    ref_buf b{out.data(), out.size() / dtype_size(dtype), dtype};
    int st = check_signature(f->tail_behavior, f->tail_spawn, &sh, sizeof sh, &b, 1);
    if (st != REF_OK) {
      resolve(sys, m.req, st, 0, {});
      return;
    }
    Msg fm;
    fm.req = m.req;
    fm.sender = (uint32_t)actor_id;
    fm.seq = f->next_seq[fm.sender]++;
    fm.args = as_bytes(std::vector<ref_shape_args>{sh});
    fm.in.push_back(std::move(out));
    fm.in_dtype.push_back(dtype);
    fm.in_numel.push_back(b.numel);
    fm.forward_to = 0;
    f->mailbox.push_back(std::move(fm));
    return;
  }
  resolve(sys, m.req, status, dtype, std::move(out));
}

extern "C" int caf_ref_become(ref_system* sys, uint64_t actor, int32_t behavior,
                              const ref_spawn_args* args) {
  Actor* a = find_actor(sys, actor);
  if (a == nullptr || !a->alive) return REF_E_NO_ACTOR;
  if (behavior < REF_BHV_NOOP || behavior > REF_BHV_FAULT) return REF_E_INVALID;
  const ref_spawn_args sp = args ? *args : ref_spawn_args{0, 0};
  if (sp.forward_to != 0) {
    Actor* f = find_actor(sys, sp.forward_to);
    if (f == nullptr || !f->alive) return REF_E_INVALID;
  }
  Msg m;
  m.req = 0;
  m.sender = 0;
  m.seq = 0;
  m.forward_to = 0;
  m.become = true;
  m.become_behavior = behavior;
  m.become_spawn = sp;
  a->mailbox.push_back(std::move(m));
  a->tail_behavior = behavior;
  a->tail_spawn = sp;
  return REF_OK;
}

extern "C" uint64_t caf_ref_run(ref_system* sys) {
  uint64_t handled = 0;
  bool any = true;
  while (any) {
    any = false;
    for (size_t i = 0; i < sys->actors.size(); ++i) {
      Actor& a = sys->actors[i];
      if (!a.alive || a.mailbox.empty()) continue;  // waiting (or done)
      Msg m = std::move(a.mailbox.front());         // ready -> running
      a.mailbox.pop_front();
      handle(sys, i + 1, m);
      handled += 1;
      any = true;
    }
  }
  return handled;
}

extern "C" int caf_ref_quit(ref_system* sys, uint64_t actor, uint32_t /*reason*/) {
  Actor* a = find_actor(sys, actor);
  if (a == nullptr || !a->alive) return REF_E_NO_ACTOR;
  a->alive = false;
  while (!a->mailbox.empty()) {
    Msg m = std::move(a->mailbox.front());
    a->mailbox.pop_front();
    resolve(sys, m.req, REF_E_QUIT, 0, {});
  }
  return REF_OK;
}

extern "C" int caf_ref_reply(ref_system* sys, uint64_t req, int32_t* status, void* out,
                             uint64_t cap, uint64_t* bytes, int32_t* dtype,
                             uint32_t* resolutions) {
  auto it = sys->replies.find(req);
  if (it == sys->replies.end()) return REF_E_INVALID;
  const Reply& r = it->second;
  if (resolutions) *resolutions = r.resolutions;
  if (!r.resolved) return 0;
  if (status) *status = r.status;
  if (dtype) *dtype = r.dtype;
  if (bytes) *bytes = r.bytes.size();
  if (out && cap) std::memcpy(out, r.bytes.data(), cap < r.bytes.size() ? cap : r.bytes.size());
  return 1;
}

extern "C" int caf_ref_timeout(ref_system* sys, uint64_t req) {
  auto it = sys->replies.find(req);
  if (it == sys->replies.end()) return REF_E_INVALID;
  if (it->second.resolved) return REF_OK;
  it->second.resolved = true;
  it->second.status = REF_E_TIMEOUT;
  // Not counted as a reply: resolutions counts replies delivered by actors.
  return REF_OK;
}

extern "C" uint64_t caf_ref_dequeue_log(ref_system* sys, uint64_t actor, uint32_t* senders,
                                        uint32_t* seqs, uint64_t cap) {
  Actor* a = find_actor(sys, actor);
  if (a == nullptr) return 0;
  uint64_t n = a->log.size();
  for (uint64_t i = 0; i < n && i < cap; ++i) {
    senders[i] = a->log[i].first;
    seqs[i] = a->log[i].second;
  }
  return n;
}

extern "C" uint64_t caf_ref_actor_state(ref_system* sys, uint64_t actor) {
  Actor* a = find_actor(sys, actor);
  return a ? a->state : 0;
}
