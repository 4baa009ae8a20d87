// Host-side scheduling of energy/force requests for continuous batching.
//
// A request is a system of n atoms and a number of successive evaluations
// (steps).  Admitted requests own a contiguous range of atom slots (their
// device coordinates and persistent neighbour lists live there) and take part
// in every iteration until their last step is launched.  Admission is
// first-come first-served: the head of the queue enters when a slot range of
// its size is free, the atoms of one iteration stay within the batch budget
// and the number of requests in flight within its limit; otherwise it, and
// everything behind it, waits.  A request that could never fit is refused at
// submission.
//
// Pure host code (no HIP calls), shared by the device server and by the
// host-only scheduler entry points, so that it runs and is tested without a
// GPU.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstddef>
#include <deque>
#include <unordered_map>
#include <utility>
#include <vector>

namespace nnp {

// First-fit allocator of contiguous ranges in [0, total).  Free ranges are
// kept sorted by start and merged with their neighbours on release.
class SlotAllocator {
 public:
  explicit SlotAllocator(int64_t total = 0) : total_(total) {
    if (total > 0) free_.push_back({0, total});
  }
  int64_t total() const { return total_; }

  // First slot of a free range of n slots, or -1.
  int64_t alloc(int64_t n) {
    for (size_t k = 0; k < free_.size(); ++k) {
      if (free_[k].second >= n) {
        const int64_t s = free_[k].first;
        if (free_[k].second == n)
          free_.erase(free_.begin() + (long)k);
        else
          free_[k] = {s + n, free_[k].second - n};
        return s;
      }
    }
    return -1;
  }

  void release(int64_t start, int64_t n) {
    size_t k = 0;
    while (k < free_.size() && free_[k].first < start) ++k;
    free_.insert(free_.begin() + (long)k, {start, n});
    // merge with the right neighbour, then the left one
    if (k + 1 < free_.size() && free_[k].first + free_[k].second == free_[k + 1].first) {
      free_[k].second += free_[k + 1].second;
      free_.erase(free_.begin() + (long)k + 1);
    }
    if (k > 0 && free_[k - 1].first + free_[k - 1].second == free_[k].first) {
      free_[k - 1].second += free_[k].second;
      free_.erase(free_.begin() + (long)k);
    }
  }

  int64_t free_slots() const {
    int64_t s = 0;
    for (auto &r : free_) s += r.second;
    return s;
  }
  const std::vector<std::pair<int64_t, int64_t>> &ranges() const { return free_; }

 private:
  int64_t total_;
  std::vector<std::pair<int64_t, int64_t>> free_;  // (start, length)
};

struct Job {
  int64_t id = 0;
  int n_atoms = 0;
  int n_steps = 0;
  double t_arrival = 0.0, t_admitted = -1.0, t_done = -1.0;
  int64_t slot = -1;
  int launched = 0;   // steps enqueued
  int completed = 0;  // steps whose results are back
  bool failed = false;  // stopped early (fail); finished, without results
};

// One request's part in a launched iteration.
struct LaunchItem {
  int64_t id;
  int64_t slot;
  int n_atoms;
  int step;    // 0-based index of the step evaluated
  bool last;   // the request's final step
};

class Scheduler {
 public:
  Scheduler(int64_t slots, int64_t max_batch_atoms, int max_active)
      : alloc_(slots), max_batch_atoms_(max_batch_atoms), max_active_(max_active) {}

  // false if the request can never run (bigger than the pool or the batch
  // budget, no steps, or a duplicate id).
  bool submit(int64_t id, int n_atoms, int n_steps, double t_arrival) {
    if (n_atoms < 1 || n_steps < 1 || n_atoms > alloc_.total() || n_atoms > max_batch_atoms_ ||
        jobs_.count(id))
      return false;
    Job j;
    j.id = id;
    j.n_atoms = n_atoms;
    j.n_steps = n_steps;
    j.t_arrival = t_arrival;
    jobs_[id] = j;
    queue_.push_back(id);
    return true;
  }

  // Admits from the head of the queue, at most max_n; returns the admitted
  // ids in order.
  std::vector<int64_t> admit(double now, size_t max_n = SIZE_MAX) {
    std::vector<int64_t> out;
    while (!queue_.empty() && out.size() < max_n) {
      Job &j = jobs_[queue_.front()];
      if ((int)active_.size() >= max_active_) break;
      if (active_atoms_ + j.n_atoms > max_batch_atoms_) break;
      const int64_t s = alloc_.alloc(j.n_atoms);
      if (s < 0) break;
      queue_.pop_front();
      j.slot = s;
      j.t_admitted = now;
      active_.push_back(j.id);
      active_atoms_ += j.n_atoms;
      out.push_back(j.id);
    }
    return out;
  }

  // The next iteration: one step of every active request, in admission order.
  // A request whose last step this is leaves the active set and its slots are
  // free for later admissions (work on one stream runs in order, so the new
  // owner's data cannot overtake this iteration).
  std::vector<LaunchItem> launch() {
    std::vector<LaunchItem> items;
    items.reserve(active_.size());
    std::vector<int64_t> keep;
    keep.reserve(active_.size());
    for (int64_t id : active_) {
      Job &j = jobs_[id];
      const bool last = j.launched + 1 == j.n_steps;
      items.push_back({id, j.slot, j.n_atoms, j.launched, last});
      ++j.launched;
      if (last) {
        alloc_.release(j.slot, j.n_atoms);
        active_atoms_ -= j.n_atoms;
      } else {
        keep.push_back(id);
      }
    }
    active_.swap(keep);
    if (!items.empty()) ++iterations_;
    for (auto &it : items) atom_evals_ += it.n_atoms;
    return items;
  }

  // Results of one step of request id are back; true when that was its last.
  bool complete(int64_t id, double now) {
    auto f = jobs_.find(id);
    if (f == jobs_.end()) return false;
    Job &j = f->second;
    ++j.completed;
    if (j.completed == j.n_steps) {
      j.t_done = now;
      return true;
    }
    return false;
  }

  // Stops a request early (its evaluation failed): it leaves the active set,
  // its slots are free for later admissions (as after its last step, work on
  // one stream runs in order) and it counts as finished.  Its steps already
  // launched stay counted.  false if it is unknown, queued or already
  // finished.
  bool fail(int64_t id, double now) {
    auto f = jobs_.find(id);
    if (f == jobs_.end()) return false;
    Job &j = f->second;
    if (j.t_admitted < 0 || j.failed || j.completed == j.n_steps) return false;
    auto a = std::find(active_.begin(), active_.end(), id);
    if (a != active_.end()) {
      active_.erase(a);
      alloc_.release(j.slot, j.n_atoms);
      active_atoms_ -= j.n_atoms;
    }
    j.failed = true;
    j.t_done = now;
    return true;
  }

  // Forgets a finished request (its record was handed out).
  void forget(int64_t id) { jobs_.erase(id); }

  const Job *job(int64_t id) const {
    auto f = jobs_.find(id);
    return f == jobs_.end() ? nullptr : &f->second;
  }
  int64_t queued() const { return (int64_t)queue_.size(); }
  int64_t active() const { return (int64_t)active_.size(); }
  int64_t active_atoms() const { return active_atoms_; }
  int64_t free_slots() const { return alloc_.free_slots(); }
  int64_t iterations() const { return iterations_; }
  int64_t atom_evals() const { return atom_evals_; }
  int64_t max_batch_atoms() const { return max_batch_atoms_; }
  int max_active() const { return max_active_; }
  const SlotAllocator &slots() const { return alloc_; }

 private:
  SlotAllocator alloc_;
  int64_t max_batch_atoms_;
  int max_active_;
  std::unordered_map<int64_t, Job> jobs_;
  std::deque<int64_t> queue_;
  std::vector<int64_t> active_;
  int64_t active_atoms_ = 0;
  int64_t iterations_ = 0;
  int64_t atom_evals_ = 0;
};

}  // namespace nnp
