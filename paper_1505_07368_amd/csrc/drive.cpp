// Native load driver: issues a list of requests through the public C ABI
// and records per-request reply latency, so benchmarks measure the actor
// runtime rather than Python call overhead.
//
//  * closed loop: at most `window` requests outstanding (window 1 is
//    ping-pong); latency = reply time - issue time.
//  * open loop: request i is issued at its scheduled arrival time; latency
//    = reply time - scheduled time, so queueing delay in admission counts
//    (no coordinated omission).
//  * host-mediated chains: each reply is re-sent by the host to the next
//    pipeline actor, the comparison point for device-side forwarding.
#include <immintrin.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/caf_gpu.h"

int64_t cafgpu_future_issue_ns(const caf_future* f);
int64_t cafgpu_future_done_ns(const caf_future* f);

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
  std::vector<Pending> pend;
  pend.reserve(window + 8);
  int first_err = CAF_OK;
  const int64_t t_start = now_ns();
  uint64_t next = 0, done = 0;

  auto issue_first = [&](uint64_t i, int64_t t_ref) -> bool {
    const caf_msg& m = msgs[i];
    const bool final_here = chain_hops == 0;
    caf_future* f = nullptr;
    int st = caf_gpu_request(sys, m.actor, m.sender, m.args, m.args_bytes, m.in, m.n_in,
                             (final_here && m.out.data) ? &m.out : nullptr, m.forward_to, &f);
    if (st != CAF_OK) {
      if (status) status[i] = st;
      if (st != CAF_E_OVERLOAD && first_err == CAF_OK) first_err = st;
      ++done;
      return false;
    }
    Pending p;
    p.f = f;
    p.idx = i;
    p.t_ref = t_ref;
    pend.push_back(p);
    return true;
  };

  // Handles a resolved entry; returns true if it stays pending (next stage).
  auto on_reply = [&](Pending& p) -> bool {
    caf_buf res{};
    int32_t rs = CAF_OK;
    caf_future_poll(p.f, &res, &rs);
    if (p.prev) {
      caf_future_release(p.prev);
      p.prev = nullptr;
    }
    if (rs == CAF_OK && p.stage < chain_hops) {
      const caf_msg& m = msgs[p.idx];
      const uint32_t n = (uint32_t)std::llround(std::sqrt((double)res.numel));
      Pending q;
      q.prev = p.f;
      q.idx = p.idx;
      q.stage = p.stage + 1;
      q.t_ref = p.t_ref;
      q.in = res;
      q.shape.rows = n;
      q.shape.cols = n;
      const bool final_here = q.stage == chain_hops;
      caf_future* f = nullptr;
      int st = caf_gpu_request(sys, hop_actor[p.stage], m.sender, &q.shape, sizeof q.shape, &q.in,
                               1, (final_here && m.out.data) ? &m.out : nullptr, 0, &f);
      if (st != CAF_OK) {
        caf_future_release(q.prev);
        if (status) status[p.idx] = st;
        if (first_err == CAF_OK) first_err = st;
        ++done;
        return false;
      }
      q.f = f;
      p = q;
      return true;
    }
    if (status) status[p.idx] = rs;
    if (latency_ns) latency_ns[p.idx] = cafgpu_future_done_ns(p.f) - p.t_ref;
    caf_future_release(p.f);
    ++done;
    return false;
  };

  auto harvest = [&]() -> bool {
    bool any = false;
    for (size_t k = 0; k < pend.size();) {
      if (caf_future_poll(pend[k].f, nullptr, nullptr) == 1) {
        any = true;
        if (on_reply(pend[k])) {
          ++k;
        } else {
          pend[k] = pend.back();
          pend.pop_back();
        }
      } else {
        ++k;
      }
    }
    return any;
  };

  if (!arrival_ns) {
    while (done < count) {
      while (next < count && pend.size() < window) {
        const int64_t t = now_ns();
        issue_first(next, t);
        if (!pend.empty() && pend.back().idx == next)
          pend.back().t_ref = cafgpu_future_issue_ns(pend.back().f);
        ++next;
      }
      if (!harvest()) _mm_pause();
    }
  } else {
    while (done < count) {
      const int64_t now = now_ns() - t_start;
      bool issued = false;
      while (next < count && arrival_ns[next] <= now && pend.size() < window) {
        issue_first(next, t_start + arrival_ns[next]);
        ++next;
        issued = true;
      }
      if (!harvest() && !issued) _mm_pause();
    }
  }
  if (elapsed_s) *elapsed_s = (double)(now_ns() - t_start) * 1e-9;
  return first_err;
}
