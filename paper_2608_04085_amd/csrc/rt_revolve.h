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
