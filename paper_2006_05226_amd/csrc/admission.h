// Admission policy of the serving loop, free of any device code so that it is
// tested on the CPU (against a mock allocator, under the address, undefined-
// behaviour and thread sanitizers) as well as used by server.cpp.
//
// * Device memory: a request is admitted only when its footprint estimate
//   fits in what the HBM budget has left; it keeps that share until release.
// * Host memory: a queued request holds host copies of its inputs (the
//   Cholesky vectors unless they are drawn on the device).  The bytes held by
//   queued requests are bounded; a request that would pass the bound is
//   refused as busy (it may be submitted again later), and one that alone
//   exceeds it is refused as too large.  The copy is dropped (drop_host) as
//   soon as the admitted request has staged its inputs on the device.
// * Order: first in, first out, with backfill: a lane takes the first queued
//   request that fits, so a large request at the head does not block smaller
//   ones behind it.
//
// Not thread safe by itself: the caller holds one mutex around every call.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>

namespace mlcc {

enum class AdmitStatus { ok, too_large_hbm, too_large_host, busy, stopped };

template <typename R> class Admission {
 public:
  struct Item {
    R *req;
    uint64_t hbm, host;
  };

  Admission(uint64_t hbm_budget, uint64_t host_budget, size_t max_queue)
      : hbm_budget_(hbm_budget), host_budget_(host_budget), max_queue_(max_queue) {}

  // Reserves the host bytes of a request before its inputs are copied, so
  // that concurrent submits cannot together pass the bound while copying.
  AdmitStatus reserve(uint64_t hbm, uint64_t host) {
    if (stopped_) return AdmitStatus::stopped;
    if (hbm > hbm_budget_) return AdmitStatus::too_large_hbm;
    if (host > host_budget_) return AdmitStatus::too_large_host;
    if (queue_.size() >= max_queue_ || host_held() + host > host_budget_) return AdmitStatus::busy;
    host_reserved_ += host;
    return AdmitStatus::ok;
  }

  // Gives back a reservation whose request is not queued after all.
  void cancel(uint64_t host) { host_reserved_ -= host; }

  // Queues a request with a reservation (its inputs are copied now); on any
  // status but ok the caller still holds the reservation and cancels it.
  AdmitStatus enqueue(R *r, uint64_t hbm, uint64_t host) {
    if (stopped_) return AdmitStatus::stopped;
    if (queue_.size() >= max_queue_) return AdmitStatus::busy;
    queue_.push_back(Item{r, hbm, host});
    host_reserved_ -= host;
    host_queued_ += host;
    return AdmitStatus::ok;
  }

  // The first queued request whose footprint fits in the HBM left, charged
  // to the budget, or nullptr.
  R *admit(uint64_t *hbm_out = nullptr, uint64_t *host_out = nullptr) {
    for (auto it = queue_.begin(); it != queue_.end(); ++it) {
      if (it->hbm <= hbm_budget_ - hbm_in_use_) {
        const Item item = *it;
        queue_.erase(it);
        hbm_in_use_ += item.hbm;
        host_admitted_ += item.host;
        host_queued_ -= item.host;
        if (hbm_out) *hbm_out = item.hbm;
        if (host_out) *host_out = item.host;
        return item.req;
      }
    }
    return nullptr;
  }

  // An admitted request no longer holds its host copy.
  void drop_host(uint64_t host) { host_admitted_ -= host; }

  // An admitted request finished: its device share is returned.
  void release(uint64_t hbm) { hbm_in_use_ -= hbm; }

  // Stops admitting; returns the requests still queued (the caller owns them).
  std::deque<Item> stop() {
    stopped_ = true;
    std::deque<Item> left;
    left.swap(queue_);
    host_queued_ = 0;
    return left;
  }

  bool stopped() const { return stopped_; }
  size_t queued() const { return queue_.size(); }
  uint64_t hbm_in_use() const { return hbm_in_use_; }
  uint64_t hbm_budget() const { return hbm_budget_; }
  uint64_t host_queued() const { return host_queued_; }
  uint64_t host_held() const { return host_reserved_ + host_queued_ + host_admitted_; }
  uint64_t host_budget() const { return host_budget_; }

 private:
  uint64_t hbm_budget_, host_budget_;
  size_t max_queue_;
  std::deque<Item> queue_;
  uint64_t hbm_in_use_ = 0, host_reserved_ = 0, host_queued_ = 0, host_admitted_ = 0;
  bool stopped_ = false;
};

}  // namespace mlcc
