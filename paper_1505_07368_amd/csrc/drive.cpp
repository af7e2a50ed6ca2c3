// Native load driver: issues a list of requests through the library's
// request path and records per-request reply latency, so benchmarks measure
// the actor runtime rather than Python call overhead.
//
//  * closed loop: at most `window` requests outstanding (window 1 is
//    ping-pong); latency = reply time - issue time.
//  * open loop: request i is issued at its scheduled arrival time; latency
//    = reply time - scheduled time, so queueing delay in admission counts
//    (no coordinated omission).
//  * host-mediated chains: each reply is re-sent by the host to the next
//    pipeline actor, the comparison point for device-side forwarding.
//
// Admission.  The driver never waits inside a request call (a request
// blocked on arena space that only the driver's own harvest would free
// could never return).  With a blocking system, a request that does not fit
// yet stays at the head of the driver's queue -- later messages keep their
// order behind it -- and is retried after the next replies are harvested,
// which frees their slots and arena buffers: messages are admitted as room
// frees up, and the open-loop latency includes that wait.  The next stage
// of a host-mediated chain waits the same way, ahead of new messages; if
// stages wait while none of the driver's own requests is in flight (the
// arena is held by the waiting chains' replies, so no wait could end), the
// oldest waiting chain is refused (CAF_E_OVERLOAD) and its reply released.
// With a non-blocking system, a refused request is final (CAF_E_OVERLOAD).
//
// Replies are harvested through a completion queue that the poller thread
// fills with the tags of resolved requests, so harvesting costs O(1) per
// reply whatever the window.
#include <immintrin.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "caf_internal.h"

namespace {

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  caf_future* f = nullptr;
  caf_future* prev = nullptr;  // previous chain stage (its reply is this stage's input)
  uint64_t idx = 0;
  uint32_t stage = 0;
  int64_t t_ref = 0;  // issue or scheduled time
  caf_buf in{};       // chain input
  caf_shape_args shape{};
};

}  // namespace

extern "C" int caf_gpu_drive(caf_gpu_system* sys, const caf_msg* msgs, uint64_t count,
                             uint32_t window, const int64_t* arrival_ns, uint32_t chain_hops,
                             const caf_actor* hop_actor, int64_t* latency_ns, int32_t* status,
                             double* elapsed_s) {
  if (!sys || (!msgs && count) || (chain_hops && !hop_actor) || chain_hops > 2)
    return CAF_E_INVALID;
  if (window == 0) window = 1;
  for (uint64_t i = 0; i < count; ++i) {
    if (latency_ns) latency_ns[i] = -1;
    if (status) status[i] = CAF_E_INVALID;
  }
  uint64_t qcap = 64;
  while (qcap < 2ull * window + 64) qcap <<= 1;
  std::vector<uint32_t> qbuf;
  std::vector<Pending> pend;
  std::vector<uint32_t> free_tags;
  try {  // no exception crosses the C ABI; nothing is issued before this
    qbuf.resize(qcap);
    pend.resize(window);
    free_tags.reserve(window);
  } catch (...) {
    return CAF_E_OVERLOAD;
  }
  cafgpu::DriveQ q;
  q.buf = qbuf.data();
  q.mask = qcap - 1;
  for (uint32_t k = 0; k < window; ++k) free_tags.push_back(window - 1 - k);
  int first_err = CAF_OK;
  uint64_t next = 0, done = 0;
  uint64_t live = 0;  // this driver's requests issued and not yet harvested
  const int64_t t_start = now_ns();

  auto fail = [&](uint64_t i, int st) {
    if (status) status[i] = st;
    if (st != CAF_E_OVERLOAD && first_err == CAF_OK) first_err = st;
    ++done;
  };

  const bool wait_for_room = cafgpu_blocking(sys);
  // Issues message i; false if it does not fit yet (blocking system only).
  auto issue_first = [&](uint64_t i, int64_t t_sched) -> bool {
    const caf_msg& m = msgs[i];
    const uint32_t tag = free_tags.back();
    caf_future* f = nullptr;
    const bool final_here = chain_hops == 0;
    const int st = cafgpu_request_tagged(sys, m.actor, m.sender, m.args, m.args_bytes, m.in,
                                         m.n_in, (final_here && m.out.data) ? &m.out : nullptr,
                                         m.forward_to, &f, &q, tag, wait_for_room);
    if (st == kTryLater) return false;
    if (st != CAF_OK) {
      fail(i, st);
      return true;
    }
    free_tags.pop_back();
    ++live;
    Pending& p = pend[tag];
    p = Pending();
    p.f = f;
    p.idx = i;
    p.t_ref = t_sched >= 0 ? t_sched : cafgpu_future_issue_ns(f);
    return true;
  };

  // Sends the next chain stage of tag k (its input: the previous stage's
  // reply); false if it does not fit yet (blocking system only).
  auto issue_hop = [&](uint32_t k) -> bool {
    Pending& p = pend[k];
    const caf_msg& m = msgs[p.idx];
    const bool final_here = p.stage == chain_hops;
    caf_future* f = nullptr;
    const int st = cafgpu_request_tagged(sys, hop_actor[p.stage - 1], m.sender, &p.shape,
                                         sizeof p.shape, &p.in, 1,
                                         (final_here && m.out.data) ? &m.out : nullptr, 0, &f,
                                         &q, k, wait_for_room);
    if (st == kTryLater) return false;
    if (st == CAF_OK) {
      p.f = f;
      ++live;
      return true;
    }
    caf_future_release(p.prev);
    p.prev = nullptr;
    fail(p.idx, st);
    free_tags.push_back(k);
    return true;
  };
  // chain stages waiting for room, in the order their inputs arrived (a
  // ring: at most `window` tags wait at once)
  std::vector<uint32_t> hop_wait;
  uint64_t hop_head = 0, hop_tail = 0;
  try {
    hop_wait.resize(chain_hops ? window : 1);
  } catch (...) {
    return CAF_E_OVERLOAD;
  }

  // Handles the resolved request of tag k.
  auto on_reply = [&](uint32_t k) {
    --live;
    Pending& p = pend[k];
    caf_buf res{};
    int32_t rs = CAF_OK;
    caf_future_poll(p.f, &res, &rs);
    if (p.prev) {
      caf_future_release(p.prev);
      p.prev = nullptr;
    }
    if (rs == CAF_OK && p.stage < chain_hops) {
      const uint32_t n = (uint32_t)std::llround(std::sqrt((double)res.numel));
      p.prev = p.f;
      p.in = res;
      p.shape.rows = n;
      p.shape.cols = n;
      p.stage += 1;
      // stages already waiting go first, so chains keep their order
      if (hop_head < hop_tail || !issue_hop(k)) hop_wait[hop_tail++ % window] = k;
      return;
    }
    if (status) status[p.idx] = rs;
    if (latency_ns) latency_ns[p.idx] = cafgpu_future_done_ns(p.f) - p.t_ref;
    caf_future_release(p.f);
    p.f = nullptr;
    ++done;
    free_tags.push_back(k);
  };

  auto harvest = [&]() -> bool {
    bool any = false;
    const uint64_t tail = __atomic_load_n(&q.tail, __ATOMIC_ACQUIRE);
    while (q.head < tail) {
      const uint32_t k = q.buf[q.head & q.mask];
      q.head += 1;
      on_reply(k);
      any = true;
    }
    return any;
  };

  while (done < count) {
    bool issued = false;
    // chain stages that did not fit go before any new message
    while (hop_head < hop_tail && issue_hop(hop_wait[hop_head % window])) {
      ++hop_head;
      issued = true;
    }
    if (hop_head < hop_tail && live == 0) {
      // Stages wait and none of this driver's requests is in flight to free
      // room: the memory is held by the waiting chains' own replies (or by
      // others), so waiting could never end.  The oldest waiting chain is
      // refused and its reply released, which lets the others go on.
      const uint32_t k = hop_wait[hop_head++ % window];
      Pending& p = pend[k];
      caf_future_release(p.prev);
      p.prev = nullptr;
      fail(p.idx, CAF_E_OVERLOAD);
      free_tags.push_back(k);
      issued = true;
    }
    // messages [next, due) may be issued now, in order
    uint64_t due = count;
    if (arrival_ns) {
      const int64_t now = now_ns() - t_start;
      due = next;
      while (due < count && arrival_ns[due] <= now) ++due;
    }
    while (next < due && !free_tags.empty() && hop_head == hop_tail) {
      if (!issue_first(next, arrival_ns ? t_start + arrival_ns[next] : -1)) break;
      ++next;
      issued = true;
    }
    if (!harvest() && !issued) _mm_pause();
  }
  if (elapsed_s) *elapsed_s = (double)(now_ns() - t_start) * 1e-9;
  return first_err;
}
