// Binomial checkpointing schedule (Griewank & Walther's "revolve"; the paper
// manages the memory of its reverse sweep with binomial checkpointing,
// Sec. 3.4).  Host code.
//
// Reversing l steps with c checkpoint slots (one of them holding the state
// at the start of the range) needs at least
//     t(l, c) = r l - beta(c + 1, r - 1)
// forward re-computations, where beta(c, r) = (c + r)! / (c! r!) and r is the
// smallest repetition number with beta(c, r) >= l.  The schedule below
// attains it: advance m steps, take a snapshot there, reverse the right part
// with c - 1 slots, then the left part with c slots, with m in
// [max(beta(c, r-2), l - beta(c-1, r)), min(beta(c, r-1), l - beta(c-1, r-1))]:
// there the right part needs repetition number exactly r and the left part
// exactly r - 1, and their costs add up to t(l, c) by Pascal's rule.  The
// window is never empty because beta(c, r-1) < l <= beta(c, r).
#pragma once
#include <algorithm>
#include <cstdint>
#include <limits>
#include <vector>

namespace rtrev {

struct Action {
  enum Kind { ADVANCE, TAKESHOT, RESTORE, REVERSE } kind;
  int to;    // ADVANCE: step index to reach
  int slot;  // TAKESHOT / RESTORE
};

inline uint64_t beta(int c, int r) {
  // C(c + r, c), saturating at 2^62
  if (c < 0 || r < 0) return 0;
  const int k = std::min(c, r);
  unsigned __int128 v = 1;
  for (int i = 1; i <= k; ++i) {
    v = v * (unsigned)(c + r - k + i) / (unsigned)i;
    if (v > ((unsigned __int128)1 << 62)) return (uint64_t)1 << 62;
  }
  return (uint64_t)v;
}

inline int repetition(int l, int c) {
  int r = 0;
  while (beta(c, r) < (uint64_t)l) ++r;
  return r;
}

// Minimal number of forward steps to reverse l steps with c slots.
inline int64_t min_forward_steps(int l, int c) {
  if (l <= 1) return 0;
  if (c <= 1) return (int64_t)l * (l - 1) / 2;
  const int r = repetition(l, c);
  return (int64_t)r * l - (int64_t)beta(c + 1, r - 1);
}

namespace detail {
inline void rev(int start, int l, int c, int slot, std::vector<int>& free_slots, std::vector<Action>& out) {
  if (l <= 0) return;
  if (l == 1) {
    out.push_back({Action::RESTORE, 0, slot});
    out.push_back({Action::REVERSE, start, 0});
    return;
  }
  if (c <= 1 || free_slots.empty()) {
    for (int k = l - 1; k >= 0; --k) {
      out.push_back({Action::RESTORE, 0, slot});
      if (k > 0) out.push_back({Action::ADVANCE, start + k, 0});
      out.push_back({Action::REVERSE, start + k, 0});
    }
    return;
  }
  const int r = repetition(l, c);
  const uint64_t a = (uint64_t)l > beta(c - 1, r) ? (uint64_t)l - beta(c - 1, r) : 1;
  const uint64_t lo = std::max<uint64_t>(a, beta(c, r - 2));
  int m = (int)std::max<uint64_t>(1, std::min<uint64_t>(lo, (uint64_t)l - 1));
  out.push_back({Action::RESTORE, 0, slot});
  out.push_back({Action::ADVANCE, start + m, 0});
  const int s2 = free_slots.back();
  free_slots.pop_back();
  out.push_back({Action::TAKESHOT, 0, s2});
  rev(start + m, l - m, c - 1, s2, free_slots, out);
  free_slots.push_back(s2);
  rev(start, m, c, slot, free_slots, out);
}
}  // namespace detail

// Schedule for reversing steps nsteps-1 .. 0 with `slots` slots; slot 0
// holds the initial state.  The working state starts at step 0.
inline std::vector<Action> schedule(int nsteps, int slots) {
  std::vector<Action> out;
  std::vector<int> free_slots;
  for (int k = slots - 1; k >= 1; --k) free_slots.push_back(k);
  detail::rev(0, nsteps, std::max(1, slots), 0, free_slots, out);
  return out;
}

// Two-level plan.  The forward march that evaluates the objective (and
// finds the step count) also leaves the state of every step k * interval in
// slot k, k < K = ceil(nsteps / interval): those snapshots cost no extra
// forward steps.  The reverse sweep then takes the segments from the last
// to the first and reverses each with the binomial schedule above, starting
// from its own snapshot and using the slots no level-1 snapshot holds plus
// those of the segments already reversed.  The returned actions are the
// reverse sweep only, with the level-1 snapshots taken as present.
inline std::vector<Action> two_level_plan(int nsteps, int interval, int slots) {
  std::vector<Action> out;
  const int K = (nsteps + interval - 1) / interval;
  std::vector<int> free_slots;
  for (int k = slots - 1; k >= K; --k) free_slots.push_back(k);
  for (int k = K - 1; k >= 0; --k) {
    const int start = k * interval, l = std::min(interval, nsteps - start);
    detail::rev(start, l, 1 + (int)free_slots.size(), k, free_slots, out);
    free_slots.push_back(k);  // its segment is done: the slot is free
  }
  return out;
}

// Forward steps of the reverse sweep of two_level_plan (the level-1 march's
// nsteps steps not included), from the closed-form optimum of each segment.
inline int64_t two_level_cost(int nsteps, int interval, int slots) {
  const int K = (nsteps + interval - 1) / interval;
  if (K > slots) return std::numeric_limits<int64_t>::max();
  int64_t t = 0;
  int nfree = slots - K;
  for (int k = K - 1; k >= 0; --k) {
    const int l = std::min(interval, nsteps - k * interval);
    t += min_forward_steps(l, 1 + nfree);
    ++nfree;
  }
  return t;
}

// Level-1 interval for a march expected to take about n_est steps: the
// cheapest by two_level_cost among those whose snapshots of margin * n_est
// steps fit in slots - 1 slots (one slot stays free).
inline int level1_interval(int n_est, int slots, double margin) {
  n_est = std::max(n_est, 1);
  const int usable = std::max(slots - 1, 1);
  const int lo = std::max(1, (int)((margin * n_est + usable - 1) / usable));
  int best = lo;
  int64_t best_cost = two_level_cost(n_est, lo, slots);
  const int hi = std::min(n_est, 64 * lo);
  for (int I = lo + 1; I <= hi; ++I) {
    const int64_t t = two_level_cost(n_est, I, slots);
    if (t < best_cost) {
      best_cost = t;
      best = I;
    }
  }
  return best;
}

// Forward steps a schedule performs (each ADVANCE from the current step).
inline int64_t count_forward(const std::vector<Action>& plan) {
  int64_t n = 0;
  int cur = 0;
  std::vector<int> slot_step(1 << 20, -1);
  slot_step[0] = 0;
  for (const Action& a : plan) {
    if (a.kind == Action::ADVANCE) {
      n += a.to - cur;
      cur = a.to;
    } else if (a.kind == Action::TAKESHOT) {
      slot_step[a.slot] = cur;
    } else if (a.kind == Action::RESTORE) {
      cur = slot_step[a.slot];
    }
  }
  return n;
}

}  // namespace rtrev
