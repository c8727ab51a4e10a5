// CPU checks of the server's arena allocator and round planner (sl1m_sched.h).
// Built and run by tests/test_sched.py with g++ (address/undefined sanitizers).
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "sl1m_sched.h"

using namespace sl1m::sched;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed at %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

static void arena_tests() {
  Arena a(1 << 20);
  size_t o1, o2, o3, o4;
  CHECK(a.alloc(1000, &o1) && o1 == 0);
  CHECK(a.alloc(256, &o2) && o2 == 1024);
  CHECK(a.alloc(5000, &o3) && o3 == 1280);
  CHECK(a.used_bytes() == 1024 + 256 + 5120);
  CHECK(a.release(o2));
  CHECK(!a.release(o2));                       // double free rejected
  CHECK(a.alloc(200, &o4) && o4 == 1024);      // first fit reuses the hole
  CHECK(a.release(o1) && a.release(o4) && a.release(o3));
  CHECK(a.used_bytes() == 0 && a.n_free_blocks() == 1 && a.largest_free() == (1u << 20));
  size_t big;
  CHECK(!a.alloc((1u << 20) + 1, &big));
  // random alloc/free keeps the free list coalesced and accounting exact
  std::mt19937 rng(7);
  std::map<size_t, size_t> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || (rng() % 3)) {
      size_t sz = 1 + rng() % 40000, off;
      if (a.alloc(sz, &off)) {
        for (auto& kv : live) CHECK(off + Arena::round_up(sz) <= kv.first || kv.first + kv.second <= off);
        live[off] = Arena::round_up(sz);
      }
    } else {
      auto it2 = live.begin();
      std::advance(it2, rng() % live.size());
      CHECK(a.release(it2->first));
      live.erase(it2);
    }
    size_t used = 0;
    for (auto& kv : live) used += kv.second;
    CHECK(a.used_bytes() == used);
  }
  for (auto& kv : live) CHECK(a.release(kv.first));
  CHECK(a.n_free_blocks() == 1);
}

// Replays the planner on random request mixes and checks, per request and
// phase: every forward item exactly once and in order, then exactly one
// reduce, then every adjoint item once, then one update + final carrying the
// right phase flags; the objective phase has no adjoint and ends the request;
// a cancelled request gets no further work.
static void planner_tests() {
  // single small request: every phase fits one round
  {
    Shape s;
    s.fwd_delta = 6; s.fwd_gauss = 2; s.adj_delta = 5; s.adj_gauss = 3;
    s.vis_blocks = 4; s.pix_blocks = 3; s.evals_per_op = 1e6; s.power_iters = 3; s.max_iter = 7;
    CHECK(rounds_alone(s, 1e9) == 3 + 7 + 1);
  }
  // random shapes and budgets, several requests at once, with a cancellation
  std::mt19937 rng(11);
  for (int trial = 0; trial < 200; ++trial) {
    const int nreq = 1 + rng() % 6;
    std::vector<Request> reqs(nreq);
    for (int i = 0; i < nreq; ++i) {
      Shape& s = reqs[i].shape;
      s.fwd_delta = rng() % 30; s.fwd_gauss = rng() % 20;
      if (s.fwd_delta + s.fwd_gauss == 0) s.fwd_delta = 1;
      s.adj_delta = rng() % 25; s.adj_gauss = rng() % 15;
      if (s.adj_delta + s.adj_gauss == 0) s.adj_gauss = 1;
      s.vis_blocks = 1 + rng() % 9; s.pix_blocks = 1 + rng() % 9;
      s.prep_blocks = rng() % 3;
      s.evals_per_op = 1e5 * (1 + rng() % 1000);
      s.power_iters = rng() % 4; s.max_iter = rng() % 6;
      reqs[i].slot = i; reqs[i].ticket = 100 + i;
      if (rng() % 2) reqs[i].share = 1e5 * (1 + rng() % 300);   // per-request share
      start_request(reqs[i]);
    }
    const double budget = 1e5 * (1 + rng() % 300);
    const int cancel_at = (rng() % 2) ? int(rng() % 5) : -1;
    const int cancel_who = int(rng() % nreq);
    std::vector<Request*> act;
    for (auto& r : reqs) act.push_back(&r);
    // per request state machine mirror
    struct M { int phase = 0; int64_t f = 0, a = 0; bool red = false, prep = false; int finals = 0; bool done = false; };
    std::vector<M> m(nreq);
    RoundPlan rp;
    int64_t round = 0;
    for (; round < 100000; ++round) {
      if (round == cancel_at) reqs[cancel_who].cancelled = true;
      bool any = false;
      for (auto& r : reqs) any |= (!r.cancelled && r.phase != P_DONE);
      if (!any) break;
      plan_round(act, budget, round, rp);
      CHECK(!rp.seg[K_FINAL].empty() || !rp.seg[K_FWD_DELTA].empty() || !rp.seg[K_FWD_GAUSS].empty() ||
            !rp.seg[K_ADJ_DELTA].empty() || !rp.seg[K_ADJ_GAUSS].empty());
      for (int ki = 0; ki < K_COUNT; ++ki) {
        const int k = kRoundOrder[ki];
        std::set<int> seen;
        for (const Segment& g : rp.seg[k]) {
          CHECK(g.begin < g.end);
          CHECK(seen.insert(g.slot).second);  // at most one segment per request per kernel
          M& st = m[g.slot];
          const Shape& s = reqs[g.slot].shape;
          CHECK(!st.done);
          CHECK(!reqs[g.slot].cancelled || round < cancel_at + 1);
          switch (k) {
            case K_PREP:
              CHECK(s.prep_blocks > 0 && !st.prep && !st.red && st.f == 0);
              CHECK(g.begin == 0 && g.end == s.prep_blocks);
              st.prep = true; break;
            case K_FWD_DELTA:
              CHECK(s.prep_blocks == 0 || st.prep);
              CHECK(!st.red && g.begin == st.f && g.end <= s.fwd_delta); st.f = g.end; break;
            case K_FWD_GAUSS:
              CHECK(s.prep_blocks == 0 || st.prep);
              CHECK(!st.red && g.begin + s.fwd_delta == st.f && g.end <= s.fwd_gauss);
              st.f = g.end + s.fwd_delta; break;
            case K_REDUCE:
              CHECK(st.f == s.fwd_delta + s.fwd_gauss && !st.red && g.begin == 0 && g.end == s.vis_blocks);
              st.red = true; break;
            case K_ADJ_DELTA:
              CHECK(st.red && g.begin == st.a && g.end <= s.adj_delta); st.a = g.end; break;
            case K_ADJ_GAUSS:
              CHECK(st.red && g.begin + s.adj_delta == st.a && g.end <= s.adj_gauss);
              st.a = g.end + s.adj_delta; break;
            case K_UPDATE: {
              const bool obj = g.flags & F_OBJECTIVE;
              CHECK(st.red && (obj ? st.a == 0 : st.a == s.adj_delta + s.adj_gauss));
              CHECK(g.begin == 0 && g.end == s.pix_blocks);
              break;
            }
            case K_FINAL: {
              CHECK(st.red && g.end - g.begin == 1);
              const bool obj = g.flags & F_OBJECTIVE;
              const int expect_phase = st.phase;
              const bool is_power = expect_phase < s.power_iters;
              const bool is_fista = !is_power && expect_phase < s.power_iters + s.max_iter;
              CHECK(((g.flags & F_POWER) != 0) == is_power);
              CHECK(((g.flags & F_FISTA) != 0) == is_fista);
              CHECK(obj == (!is_power && !is_fista));
              CHECK(((g.flags & F_LAST_POWER) != 0) == (is_power && expect_phase + 1 == s.power_iters));
              st.phase++; st.f = 0; st.a = 0; st.red = false; st.prep = false;
              if (obj) st.done = true;
              break;
            }
          }
        }
      }
    }
    CHECK(round < 100000);
    for (int i = 0; i < nreq; ++i) {
      const Shape& s = reqs[i].shape;
      if (reqs[i].cancelled) continue;
      CHECK(m[i].done && m[i].phase == s.power_iters + s.max_iter + 1);
      CHECK(reqs[i].phase == P_DONE && reqs[i].done_round >= 0);
    }
  }
}

int main() {
  arena_tests();
  planner_tests();
  std::printf("sched OK\n");
  return 0;
}
