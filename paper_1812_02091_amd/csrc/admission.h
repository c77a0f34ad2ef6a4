// Admission policy of the serving engine (continuous batching), kept free of
// device code so that it runs under a fake executor on the host.
//
// The device memory budget is split at start into K launch lanes, each with
// buffers for up to B queries and W words (tables, distance rows, candidate
// lists).  Queries wait in one FIFO.  Whenever a lane is free and queries
// wait, the lane takes the FIFO's head queries -- as many as fit its B slots
// and W words -- and launches at once: a query never waits for a batch to
// fill or for a fixed lane to drain; queries that arrive while other
// batches run join the next free lane, and up to K batches run on the device
// side by side.  The head of the FIFO always fits an empty lane (submission
// rejects a query longer than W words), so no query starves and queries
// start in submission order.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace lcemd_serve {

template <typename Q>  // Q: a queued query, with a `words` member
class Admission {
 public:
  Admission(int lanes, int slots, int words) : slots_(slots), words_(words), busy_(lanes, 0) {}

  int lanes() const { return (int)busy_.size(); }
  int slots() const { return slots_; }
  int words() const { return words_; }
  bool fits(int w) const { return w >= 1 && w <= words_; }
  size_t waiting() const { return fifo_.size(); }
  bool busy(int lane) const { return busy_[lane] != 0; }
  int busy_lanes() const {
    int c = 0;
    for (char b : busy_) c += b ? 1 : 0;
    return c;
  }

  // queue a query (callers check fits() first)
  void push(Q q) { fifo_.push_back(std::move(q)); }
  Q& front() { return fifo_.front(); }
  std::deque<Q>& queue() { return fifo_; }

  // The next launch: a free lane (the lowest index) and the FIFO head's
  // queries that fit it; -1 if no lane is free or nothing waits.
  int next(std::vector<Q>& batch) {
    batch.clear();
    if (fifo_.empty()) return -1;
    int lane = -1;
    for (int i = 0; i < (int)busy_.size(); ++i)
      if (!busy_[i]) {
        lane = i;
        break;
      }
    if (lane < 0) return -1;
    int w = 0;
    while (!fifo_.empty() && (int)batch.size() < slots_ && w + fifo_.front().words <= words_) {
      w += fifo_.front().words;
      batch.push_back(std::move(fifo_.front()));
      fifo_.pop_front();
    }
    busy_[lane] = 1;
    return lane;
  }

  void done(int lane) { busy_[lane] = 0; }

 private:
  int slots_, words_;
  std::vector<char> busy_;
  std::deque<Q> fifo_;
};

}  // namespace lcemd_serve

namespace lcemd_serve {

// Slots per lane that the budget allows: lanes x slots x per-query bytes
// (plus the per-lane fixed bytes) within budget, at most max_slots; 0 when
// the budget holds no query.
inline int plan_slots(int64_t budget, double per_query_bytes, double per_lane_bytes, int lanes, int max_slots) {
  const double room = (double)budget / lanes - per_lane_bytes;
  if (room < per_query_bytes || max_slots < 1) return 0;
  const double fit = room / per_query_bytes;
  return fit >= (double)max_slots ? max_slots : (int)fit;
}

}  // namespace lcemd_serve
