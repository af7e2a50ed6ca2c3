// CPU actors and the CPU+GPU split of one Mandelbrot image (Sec. 7.5).
//
// The paper's offload experiment computes one image partly on CPU actors
// and partly on a GPU compute actor and times the whole image as the GPU's
// share grows from 0 to 100%.  This file holds the CPU actors' kernel, a pool
// of worker threads that plays the CPU actors (created on first use, kept by
// the system until caf_gpu_shutdown) and the call that runs one split.  The
// GPU share goes through the ordinary request path; nothing here is used by
// it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "caf_internal.h"

namespace {

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool args_ok(const caf_mandel_args* a) {
  return a && a->width && a->height && a->max_iter >= 1 && a->max_iter <= 65535 &&
         (a->fp == CAF_F32 || a->fp == CAF_F64);
}

// Escape counts of global rows [r0, r1), in precision T with every operation
// rounded to T and no contraction (the build forbids it): c is sampled as
// re_min + x*step_re + i*(im_min + y*step_im), |z|^2 > 4 ends the orbit.
template <typename T>
void rows_T(const caf_mandel_args& a, uint32_t r0, uint32_t r1, uint16_t* out) {
  const T re_min = (T)a.re_min, im_min = (T)a.im_min;
  const T step_re = (T)a.step_re, step_im = (T)a.step_im;
  const T four = (T)4;
  for (uint32_t y = r0; y < r1; ++y) {
    const T ci = im_min + (T)y * step_im;
    uint16_t* o = out + (uint64_t)(y - r0) * a.width;
    for (uint32_t x = 0; x < a.width; ++x) {
      const T cr = re_min + (T)x * step_re;
      T zr = 0, zi = 0;
      uint32_t n = 0;
      while (n < a.max_iter) {
        const T zr2 = zr * zr, zi2 = zi * zi;
        if (zr2 + zi2 > four) break;
        const T t = zr * zi;
        zi = (t + t) + ci;
        zr = (zr2 - zi2) + cr;
        ++n;
      }
      o[x] = (uint16_t)n;
    }
  }
}

void rows(const caf_mandel_args& a, uint32_t r0, uint32_t r1, uint16_t* out) {
  if (a.fp == CAF_F64) rows_T<double>(a, r0, r1, out);
  else rows_T<float>(a, r0, r1, out);
}

}  // namespace

namespace cafgpu {

// The CPU actors: worker threads that take rows of the current job in
// small groups (dynamic, so uneven rows balance) until none is left.
struct CpuPool {
  static constexpr uint32_t kGrab = 4;  // rows per claim
  explicit CpuPool(uint32_t n) : nthreads(n) {
    try {
      for (uint32_t i = 0; i < n; ++i) th.emplace_back([this] { work(); });
    } catch (...) {
      stop_all();  // the threads already started must be joined before unwinding
      throw;
    }
  }
  ~CpuPool() { stop_all(); }
  void stop_all() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto& t : th) t.join();
    th.clear();
  }
  // Starts rows [r0, r1) of `a` into out (row r0 first); returns at once.
  void post(const caf_mandel_args& a, uint32_t r0, uint32_t r1, uint16_t* out) {
    std::lock_guard<std::mutex> g(mu);
    job = a;
    jr0 = r0;
    jr1 = r1;
    jout = out;
    next.store(r0, std::memory_order_relaxed);
    busy = nthreads;
    ++gen;
    cv.notify_all();
  }
  void wait() {
    std::unique_lock<std::mutex> g(mu);
    done_cv.wait(g, [this] { return busy == 0; });
  }
  void work() {
    uint64_t seen = 0;
    for (;;) {
      caf_mandel_args a;
      uint32_t r1;
      uint16_t* out;
      uint32_t r0;
      {
        std::unique_lock<std::mutex> g(mu);
        cv.wait(g, [&] { return stop || gen != seen; });
        if (stop) return;
        seen = gen;
        a = job;
        r0 = jr0;
        r1 = jr1;
        out = jout;
      }
      for (;;) {
        const uint32_t r = next.fetch_add(kGrab, std::memory_order_relaxed);
        if (r >= r1) break;
        rows(a, r, std::min(r1, r + kGrab), out + (uint64_t)(r - r0) * a.width);
      }
      std::lock_guard<std::mutex> g(mu);
      if (--busy == 0) done_cv.notify_all();
    }
  }
  const uint32_t nthreads;
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  uint64_t gen = 0;
  caf_mandel_args job{};
  uint32_t jr0 = 0, jr1 = 0, busy = 0;
  uint16_t* jout = nullptr;
  std::atomic<uint32_t> next{0};
};

void cpu_pool_destroy(CpuPool* p) { delete p; }

// Staging for caf_offload_mandel_noalloc: the GPU share's replies land here
// instead of in a caller's buffer.  Every device the library runs on holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address: the address of each device's copy is looked up once,
// with that device current, and kept in offload_stage_ptr.
static __device__ __align__(256) uint16_t offload_stage[kOffloadStageBytes / sizeof(uint16_t)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex stage_mu;
void* stage_ptr[kMaxDevices] = {};
}  // namespace

int offload_stage_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return CAF_E_INVALID;
  std::lock_guard<std::mutex> g(stage_mu);
  if (stage_ptr[device]) return CAF_OK;
  void* p = nullptr;
  // the caller (caf_gpu_init) has made `device` current
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(offload_stage)) != hipSuccess || !p)
    return CAF_E_DEVICE;
  stage_ptr[device] = p;
  return CAF_OK;
}

static uint16_t* offload_stage_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(stage_mu);
  return static_cast<uint16_t*>(stage_ptr[device]);
}

}  // namespace cafgpu

using cafgpu::CpuPool;
using cafgpu::kOffloadNoallocMaxTiles;
using cafgpu::kOffloadStageBytes;

constexpr uint32_t kMaxCpuThreads = 1024;
constexpr uint32_t kOffloadTileRows = 64;  // rows per GPU request of a split

extern "C" int caf_cpu_mandel_rows(const caf_mandel_args* a, uint32_t row_begin, uint32_t row_end,
                                   uint16_t* out_host) {
  if (!args_ok(a) || !out_host || row_begin > row_end || row_end > a->height)
    return CAF_E_INVALID;
  rows(*a, row_begin, row_end, out_host);
  return CAF_OK;
}

namespace {

// One split.  stage: device memory for the GPU share's replies.
// may_start_pool: whether the CPU actors' pool may be (re)created here.
// tile_args / futs: room for ceil(gpu_rows / 64) entries.
int offload_run(caf_gpu_system* sys, caf_actor gpu_actor, const caf_mandel_args* image,
                uint32_t gpu_rows, uint32_t cpu_threads, uint16_t* stage, uint16_t* out_host,
                caf_offload_times* times, bool may_start_pool, caf_mandel_args* tile_args,
                caf_future** futs) {
  const uint32_t width = image->width, height = image->height;
  std::lock_guard<std::mutex> one_at_a_time(cafgpu::offload_mu_of(sys));
  CpuPool*& pool = cafgpu::cpu_pool_of(sys);
  if (gpu_rows < height && (!pool || pool->nthreads != cpu_threads)) {
    if (!may_start_pool) return CAF_E_INVALID;
    delete pool;
    pool = nullptr;
    try {
      pool = new CpuPool(cpu_threads);
    } catch (...) {  // no exception crosses the C ABI
      return CAF_E_OVERLOAD;
    }
  }
  const int64_t t0 = now_ns();
  if (gpu_rows < height) pool->post(*image, gpu_rows, height, out_host + (uint64_t)gpu_rows * width);
  // The GPU share: requests of at most kOffloadTileRows rows, replies into stage.
  int rc = CAF_OK;
  int64_t t_gpu = t0;
  if (gpu_rows) {
    uint32_t nf = 0;
    for (uint32_t r = 0; r < gpu_rows; r += kOffloadTileRows) {
      caf_mandel_args& ta = tile_args[nf];
      ta = *image;
      ta.row0 = r;
      ta.rows = std::min(kOffloadTileRows, gpu_rows - r);
      caf_buf out{stage + (uint64_t)r * width, (uint64_t)ta.rows * width, CAF_U16, 1};
      caf_future* f = nullptr;
      const int st = caf_gpu_request(sys, gpu_actor, 0, &ta, sizeof ta, nullptr, 0, &out, 0, &f);
      if (st != CAF_OK) {
        rc = st;
        break;
      }
      futs[nf++] = f;
    }
    for (uint32_t i = 0; i < nf; ++i) {
      caf_buf res{};
      int32_t st = CAF_OK;
      if (caf_future_wait(futs[i], -1, &res, &st) != CAF_OK) st = CAF_E_TIMEOUT;
      if (st != CAF_OK && rc == CAF_OK) rc = st;
      caf_future_release(futs[i]);
    }
    if (rc == CAF_OK &&
        hipMemcpy(out_host, stage, (uint64_t)gpu_rows * width * sizeof(uint16_t),
                  hipMemcpyDeviceToHost) != hipSuccess)
      rc = CAF_E_DEVICE;
    t_gpu = now_ns();
  }
  int64_t t_cpu = t0;
  if (gpu_rows < height) {
    pool->wait();
    t_cpu = now_ns();
  }
  if (times) {
    const int64_t t1 = now_ns();
    times->total_ns = t1 - t0;
    times->gpu_done_ns = t_gpu - t0;
    times->cpu_done_ns = t_cpu - t0;
  }
  return rc;
}

}  // namespace

extern "C" int caf_offload_mandel(caf_gpu_system* sys, caf_actor gpu_actor,
                                  const caf_mandel_args* image, uint32_t gpu_rows,
                                  uint32_t cpu_threads, uint16_t* dev_stage, uint16_t* out_host,
                                  caf_offload_times* times) {
  if (!sys || !args_ok(image) || image->row0 != 0 || image->rows != image->height ||
      gpu_rows > image->height || !out_host || (gpu_rows && !dev_stage))
    return CAF_E_INVALID;
  if (cpu_threads > kMaxCpuThreads) return CAF_E_INVALID;
  if (cpu_threads == 0) cpu_threads = std::max(1u, std::thread::hardware_concurrency());
  const uint32_t ntiles = (gpu_rows + kOffloadTileRows - 1) / kOffloadTileRows;
  std::vector<caf_mandel_args> targs(ntiles);
  std::vector<caf_future*> futs(ntiles);
  return offload_run(sys, gpu_actor, image, gpu_rows, cpu_threads, dev_stage, out_host, times,
                     true, targs.data(), futs.data());
}

extern "C" int caf_offload_mandel_noalloc(caf_gpu_system* sys, caf_actor gpu_actor,
                                          const caf_mandel_args* image, uint32_t gpu_rows,
                                          uint32_t cpu_threads, uint16_t* out_host,
                                          caf_offload_times* times) {
  if (!sys || !args_ok(image) || image->row0 != 0 || image->rows != image->height ||
      gpu_rows > image->height || !out_host)
    return CAF_E_INVALID;
  if (cpu_threads > kMaxCpuThreads) return CAF_E_INVALID;
  if (cpu_threads == 0) cpu_threads = std::max(1u, std::thread::hardware_concurrency());
  // the limits of the fixed staging array and of the on-stack request table
  if ((uint64_t)gpu_rows * image->width * sizeof(uint16_t) > kOffloadStageBytes ||
      gpu_rows > kOffloadNoallocMaxTiles * kOffloadTileRows)
    return CAF_E_INVALID;
  uint16_t* stage = cafgpu::offload_stage_ptr(cafgpu::device_of(sys));
  if (!stage) return CAF_E_DEVICE;
  caf_mandel_args targs[kOffloadNoallocMaxTiles];
  caf_future* futs[kOffloadNoallocMaxTiles];
  return offload_run(sys, gpu_actor, image, gpu_rows, cpu_threads, stage, out_host, times,
                     false, targs, futs);
}
