// Host-side scheduling for the SL1M server: an HBM arena allocator and the
// planner that decides, for every round, which work items of which active
// request go into each batched kernel.  Pure C++ (no HIP), so it is unit-tested
// on the CPU.
//
// A request's solve is the sequence of phases
//   POWER step 0 .. P-1  (only when no L is given),
//   FISTA iteration 1 .. K,
//   OBJECTIVE (forward on the final image, objective terms, output copy).
// Every phase is "[prep] -> forward items -> reduce -> adjoint items -> update
// -> final" (OBJECTIVE has no adjoint; prep, which builds per-call records from
// the phase's input vector, only for requests that need it).  Kernels of one round run in that order, so a
// request may cover a whole phase in one round when its work fits the per-round
// budget; larger requests spread the forward and adjoint items of a phase over
// several rounds.  A request never starts a new phase in the round that
// finishes the previous one (the next forward needs the update's output).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace sl1m {
namespace sched {

// First-fit allocator over [0, size) with 256-byte granules and coalescing.
class Arena {
 public:
  explicit Arena(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    free_.clear();
    used_.clear();
    size_ = size / kAlign * kAlign;
    if (size_) free_[0] = size_;
  }
  static size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  bool alloc(size_t bytes, size_t* off) {
    const size_t need = round_up(bytes > 0 ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const size_t o = it->first, rest = it->second - need;
        free_.erase(it);
        if (rest) free_[o + need] = rest;
        used_[o] = need;
        *off = o;
        return true;
      }
    }
    return false;
  }
  bool release(size_t off) {
    auto it = used_.find(off);
    if (it == used_.end()) return false;
    size_t o = off, n = it->second;
    used_.erase(it);
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && nx->first == o + n) {
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == o) {
        o = pv->first;
        n += pv->second;
        free_.erase(pv);
      }
    }
    free_[o] = n;
    return true;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  size_t used_bytes() const {
    size_t u = 0;
    for (auto& f : used_) u += f.second;
    return u;
  }
  size_t size() const { return size_; }
  size_t n_free_blocks() const { return free_.size(); }

  static constexpr size_t kAlign = 256;

 private:
  size_t size_ = 0;
  std::map<size_t, size_t> free_, used_;
};

enum Kernel {
  K_FWD_DELTA = 0, K_FWD_GAUSS, K_REDUCE, K_ADJ_DELTA, K_ADJ_GAUSS, K_UPDATE, K_FINAL, K_PREP,
  K_COUNT
};

// Order in which the kernels of one round run.
constexpr Kernel kRoundOrder[K_COUNT] = {K_PREP,      K_FWD_DELTA, K_FWD_GAUSS, K_REDUCE,
                                         K_ADJ_DELTA, K_ADJ_GAUSS, K_UPDATE,    K_FINAL};

// Segment flags (what the batched kernels do for the segment's request).
enum : int32_t {
  F_POWER = 1,        // power-iteration phase
  F_FISTA = 2,        // FISTA iteration
  F_OBJECTIVE = 4,    // final objective / output phase
  F_LAST_POWER = 8,   // last power step: derive L and start FISTA
};

enum Phase { P_POWER = 0, P_FISTA, P_OBJECTIVE, P_DONE };

// Work-item counts of one request, fixed by its plan.
struct Shape {
  int64_t fwd_delta = 0, fwd_gauss = 0;  // forward items
  int64_t adj_delta = 0, adj_gauss = 0;  // adjoint items
  int64_t vis_blocks = 0;                // reduce items
  int64_t pix_blocks = 0;                // update items
  int64_t prep_blocks = 0;               // prep items at the start of each forward (0 = none)
  double evals_per_op = 0;               // N_p * N_v
  int32_t power_iters = 0;               // 0 when L is given
  int32_t max_iter = 0;
};

struct Segment {
  int32_t slot;
  int32_t flags;
  int64_t begin, end;
};

struct Request {
  uint64_t ticket = 0;
  int slot = -1;
  Shape shape;
  Phase phase = P_POWER;
  int32_t step = 0;          // power step or FISTA iteration (0-based) within the phase
  bool in_adjoint = false;   // forward items of the current phase are all scheduled
  int64_t cursor = 0;        // next forward or adjoint item
  bool cancelled = false;
  int64_t last_round = -1;   // last round that used the request's memory
  int64_t done_round = -1;   // round whose completion finishes the request
  int32_t phases_run = 0;
  double share = 0;          // operator evals this request may take per round (0: the round's budget)
};

struct RoundPlan {
  std::vector<Segment> seg[K_COUNT];
  std::vector<uint64_t> finishing;  // tickets whose OBJECTIVE completes in this round
  double evals = 0;                 // operator evals scheduled this round
  void clear() {
    for (auto& v : seg) v.clear();
    finishing.clear();
    evals = 0;
  }
};

inline void start_request(Request& r) {
  r.phase = r.shape.power_iters > 0 ? P_POWER : P_FISTA;
  if (r.phase == P_FISTA && r.shape.max_iter == 0) r.phase = P_OBJECTIVE;
  r.step = 0;
  r.in_adjoint = false;
  r.cursor = 0;
}

inline int32_t phase_flags(const Request& r) {
  switch (r.phase) {
    case P_POWER:
      return F_POWER | (r.step + 1 == r.shape.power_iters ? F_LAST_POWER : 0);
    case P_FISTA:
      return F_FISTA;
    default:
      return F_OBJECTIVE;
  }
}

inline void advance_phase(Request& r) {
  r.in_adjoint = false;
  r.cursor = 0;
  ++r.phases_run;
  if (r.phase == P_POWER) {
    if (++r.step >= r.shape.power_iters) {
      r.phase = r.shape.max_iter > 0 ? P_FISTA : P_OBJECTIVE;
      r.step = 0;
    }
  } else if (r.phase == P_FISTA) {
    if (++r.step >= r.shape.max_iter) {
      r.phase = P_OBJECTIVE;
      r.step = 0;
    }
  } else if (r.phase == P_OBJECTIVE) {
    r.phase = P_DONE;
  }
}

// Adds item range [a, b) of a forward (or adjoint) sweep whose first `nd`
// items are delta items and the rest Gaussian items.
inline void add_seg(RoundPlan& rp, Kernel k, int32_t slot, int32_t flags, int64_t a, int64_t b) {
  if (b > a) rp.seg[k].push_back(Segment{slot, flags, a, b});
}

inline void add_split(RoundPlan& rp, Kernel kd, Kernel kg, int32_t slot, int32_t flags, int64_t nd,
                      int64_t a, int64_t b) {
  if (a < nd) add_seg(rp, kd, slot, flags, a, std::min(b, nd));
  if (b > nd) add_seg(rp, kg, slot, flags, std::max(a, nd) - nd, b - nd);
}

// Plans one round: every active (not cancelled, not done) request advances
// by at most its `share` (or `budget` when the share is 0) operator evals, at
// least one item, never past the end of its current phase.
inline void plan_round(std::vector<Request*>& active, double budget, int64_t round,
                       RoundPlan& rp) {
  rp.clear();
  for (Request* r : active) {
    if (r->cancelled || r->phase == P_DONE) continue;
    const Shape& s = r->shape;
    const int32_t fl = phase_flags(*r);
    const int64_t nf = s.fwd_delta + s.fwd_gauss;
    const int64_t na = s.adj_delta + s.adj_gauss;
    const double ev_f = nf > 0 ? s.evals_per_op / static_cast<double>(nf) : 0.0;
    const double ev_a = na > 0 ? s.evals_per_op / static_cast<double>(na) : 0.0;
    double left = r->share > 0 ? r->share : budget;
    r->last_round = round;
    if (!r->in_adjoint) {
      if (r->cursor == 0 && s.prep_blocks > 0) add_seg(rp, K_PREP, r->slot, fl, 0, s.prep_blocks);
      int64_t take = nf - r->cursor;
      if (ev_f > 0) take = std::min<int64_t>(take, std::max<int64_t>(1, static_cast<int64_t>(left / ev_f)));
      if (take > 0) {
        add_split(rp, K_FWD_DELTA, K_FWD_GAUSS, r->slot, fl, s.fwd_delta, r->cursor,
                  r->cursor + take);
        r->cursor += take;
        left -= take * ev_f;
        rp.evals += take * ev_f;
      }
      if (r->cursor < nf) continue;  // forward not finished: rest next round
      add_seg(rp, K_REDUCE, r->slot, fl, 0, s.vis_blocks);
      if (r->phase == P_OBJECTIVE) {
        add_seg(rp, K_UPDATE, r->slot, fl, 0, s.pix_blocks);
        add_seg(rp, K_FINAL, r->slot, fl, 0, 1);
        rp.finishing.push_back(r->ticket);
        r->done_round = round;
        advance_phase(*r);
        continue;
      }
      r->in_adjoint = true;
      r->cursor = 0;
      if (left <= 0 && na > 0) continue;
    }
    int64_t take = na - r->cursor;
    if (ev_a > 0) take = std::min<int64_t>(take, std::max<int64_t>(1, static_cast<int64_t>(left / ev_a)));
    if (take > 0) {
      add_split(rp, K_ADJ_DELTA, K_ADJ_GAUSS, r->slot, fl, s.adj_delta, r->cursor, r->cursor + take);
      r->cursor += take;
      rp.evals += take * ev_a;
    }
    if (r->cursor < na) continue;
    add_seg(rp, K_UPDATE, r->slot, fl, 0, s.pix_blocks);
    add_seg(rp, K_FINAL, r->slot, fl, 0, 1);
    advance_phase(*r);
  }
}

// Number of rounds a request alone needs (for tests and estimates).
inline int64_t rounds_alone(const Shape& s, double budget) {
  Request r;
  r.shape = s;
  r.slot = 0;
  start_request(r);
  std::vector<Request*> a{&r};
  RoundPlan rp;
  int64_t n = 0;
  while (r.phase != P_DONE && n < (int64_t{1} << 40)) plan_round(a, budget, n++, rp);
  return n;
}

}  // namespace sched
}  // namespace sl1m
