// Host-side replay of the band wavefront schedule (csrc/schedule.hpp) under stream and
// event semantics, for the test suite (built with g++ by tests/test_schedule.py).
//
// Model: a stream runs its launches in order; record(e, s) makes event e stand for
// everything enqueued on s so far; wait(s, e) makes later launches on s wait for what
// e stood for when the wait was enqueued.  Happens-before is tracked with a vector clock
// of two entries (one per stream).
//
// Checks, for every (rows, R) given:
//   1. any two launches that touch the same data, at least one writing it, are ordered;
//   2. every update term (target row k, source row r, column j), k < r <= j, is applied
//      by exactly one update launch;
//   3. a source row is solved before any update reads it, every update of a row is done
//      before that row is solved, and the updates of a tile come in descending source
//      order.
// Data: Z tile (k, j) (the mantissas, exponents and norms of its segments) and the W
// slot of each source row (2R slots reused cyclically).
// Usage: sched_check rows R [drop [split]]   (drop = index of a wait to omit: the result
// shows whether the checks notice; -1 = none).  Prints "OK" or the first violation.
//        sched_check batch rows R steps cr [drop]   the batch lock-step schedule
// (batch_band_schedule) as one pencil of `rows` tile rows sees it inside a group whose
// largest pencil has `steps` bands, U2 in launches of cr rows (0: one launch).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "schedule.hpp"

struct Op {
  int kind;      // 0 pre-processing, 1 solve, 2 update, 3 consolidation (both touch every tile)
  int stream;
  int vc[2];     // vector clock after this launch
  int k_lo, k_hi, j_lo, s_lo, s_hi;   // update; solve i: k_lo = i
};

struct Replay {
  int rows, R, drop;
  int nwait = 0;
  int cur[2][2] = {{0, 0}, {0, 0}};
  int ev[4][2] = {};
  std::vector<Op> ops;
  void launch(Op o) {
    cur[o.stream][o.stream] += 1;
    o.vc[0] = cur[o.stream][0];
    o.vc[1] = cur[o.stream][1];
    ops.push_back(o);
  }
  bool solve(int i, int s) {
    launch(Op{1, s, {0, 0}, i, i + 1, i, i, i});
    return true;
  }
  bool update(int k_lo, int k_hi, int j_lo, int s_lo, int s_hi, int s) {
    if (k_hi <= k_lo || j_lo >= rows) return true;   // nothing launched
    launch(Op{2, s, {0, 0}, k_lo, k_hi, j_lo, s_lo, s_hi});
    return true;
  }
  // a fused C(b) is the same steps in one launch: on one stream with nothing between them
  bool chain(int r_lo, int r_hi, int s) { return rgev::chain_steps(r_lo, r_hi, s, *this); }
  // the batch schedule's parts, in this pencil's rows (band b = B - 1 - t)
  int B = 0;
  bool band_of(int t, int& r_lo, int& r_hi) const {
    const int b = B - 1 - t;
    if (b < 0) return false;
    r_lo = R * b;
    r_hi = r_lo + R - 1 < rows - 1 ? r_lo + R - 1 : rows - 1;
    return true;
  }
  bool solve(int t, int io, int s) {
    int r_lo, r_hi;
    if (band_of(t, r_lo, r_hi) && r_hi - io >= r_lo) solve(r_hi - io, s);
    return true;
  }
  bool inband(int t, int io, int s) {
    int r_lo, r_hi;
    if (band_of(t, r_lo, r_hi) && r_hi - io > r_lo) update(r_lo, r_hi - io, r_hi - io, r_hi - io, r_hi - io, s);
    return true;
  }
  bool next(int t, int s) {
    int r_lo, r_hi;
    if (band_of(t, r_lo, r_hi) && r_lo > 0) update(r_lo - R > 0 ? r_lo - R : 0, r_lo, r_lo, r_lo, r_hi, s);
    return true;
  }
  bool above(int t, int off, int cnt, int s) {
    int r_lo, r_hi;
    if (!band_of(t, r_lo, r_hi)) return true;
    const int hi = r_lo - R - off;
    if (hi > 0) update(hi - cnt > 0 ? hi - cnt : 0, hi, r_lo, r_lo, r_hi, s);
    return true;
  }
  bool record(int e, int s) {
    ev[e][0] = cur[s][0];
    ev[e][1] = cur[s][1];
    return true;
  }
  bool wait(int s, int e) {
    if (nwait++ == drop) return true;
    for (int t = 0; t < 2; ++t)
      if (ev[e][t] > cur[s][t]) cur[s][t] = ev[e][t];
    return true;
  }
};

static bool hb(const Op& x, const Op& y) { return x.vc[x.stream] <= y.vc[x.stream]; }

static std::string desc(const Op& o) {
  char b[128];
  if (o.kind == 0 || o.kind == 3) snprintf(b, sizeof b, "%s@%c", o.kind ? "consolidate" : "preprocess", "AB"[o.stream]);
  else if (o.kind == 1) snprintf(b, sizeof b, "solve(%d)@%c", o.k_lo, "AB"[o.stream]);
  else snprintf(b, sizeof b, "update(rows %d..%d, cols >= %d, src %d..%d)@%c", o.k_lo, o.k_hi - 1, o.j_lo, o.s_lo,
                o.s_hi, "AB"[o.stream]);
  return b;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  Replay rp;
  const bool batch = std::string(argv[1]) == "batch";
  const int a0 = batch ? 2 : 1;
  if (argc < a0 + 2 || (batch && argc < 6)) return 2;
  rp.rows = atoi(argv[a0]);
  rp.R = atoi(argv[a0 + 1]);
  // pre-processing before and consolidation after, on the caller's stream
  rp.launch(Op{0, 0, {0, 0}, 0, rp.rows, 0, 0, rp.rows - 1});
  if (batch) {
    const int steps = atoi(argv[4]), cr = atoi(argv[5]);
    rp.drop = argc > 6 ? atoi(argv[6]) : -1;
    rp.B = (rp.rows + rp.R - 1) / rp.R;
    if (steps < rp.B) return 2;
    // the group's largest U2 row count per step: the largest pencil's (B = steps)
    std::vector<int> above(steps);
    for (int t = 0; t < steps; ++t) above[t] = rp.R * (steps - 2 - t) > 0 ? rp.R * (steps - 2 - t) : 0;
    std::vector<int> crs(steps, cr);
    rgev::batch_band_schedule(steps, rp.R, crs.data(), above.data(), rp);
  } else {
    rp.drop = argc > 3 ? atoi(argv[3]) : -1;
    const int split = argc > 4 ? atoi(argv[4]) : 0;
    rgev::band_schedule(rp.rows, rp.R, split, rp);
  }
  rp.launch(Op{3, 0, {0, 0}, 0, rp.rows, 0, 0, rp.rows - 1});
  const int rows = rp.rows, R = rp.R, WS = 2 * R;
  const std::vector<Op>& ops = rp.ops;
  const int n = (int)ops.size();
  auto zrect = [&](const Op& o, int& k0, int& k1, int& j0) {
    k0 = o.k_lo; k1 = o.k_hi; j0 = o.j_lo;   // Z tiles [k0, k1) x [j0, rows)
  };
  auto wslots = [&](const Op& o) {   // bit mask of W slots: written by a solve, read by an update
    unsigned msk = 0;
    if (o.kind == 0 || o.kind == 3) msk = ~0u;
    else if (o.kind == 1) msk = 1u << (o.k_lo % WS);
    else
      for (int s = o.s_lo; s <= o.s_hi && s < rows; ++s) msk |= 1u << (s % WS);
    return msk;
  };
  // 1. conflicting launches are ordered (enqueue order is the only possible direction)
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b) {
      const Op &x = ops[a], &y = ops[b];
      int xk0, xk1, xj0, yk0, yk1, yj0;
      zrect(x, xk0, xk1, xj0);
      zrect(y, yk0, yk1, yj0);
      const bool zc = xk0 < yk1 && yk0 < xk1;   // row ranges meet; column ranges always meet
      const bool wc = (x.kind != 2 || y.kind != 2) && (wslots(x) & wslots(y));
      if ((zc || wc) && !hb(x, y)) {
        printf("RACE %s | %s\n", desc(x).c_str(), desc(y).c_str());
        return 1;
      }
    }
  // 2. and 3.
  std::vector<int> solved_at(rows, -1);
  for (int a = 0; a < n; ++a)
    if (ops[a].kind == 1) solved_at[ops[a].k_lo] = a;
  for (int i = 0; i < rows; ++i)
    if (solved_at[i] < 0) {
      printf("MISSING solve(%d)\n", i);
      return 1;
    }
  for (int k = 0; k < rows; ++k)
    for (int j = k + 1; j < rows; ++j) {
      int last_src = rows;   // sources of tile (k, j) must come in descending order
      std::vector<int> cover(rows, 0);
      for (int a = 0; a < n; ++a) {
        const Op& o = ops[a];
        if (o.kind != 2 || k < o.k_lo || k >= o.k_hi || j < o.j_lo) continue;
        int hi = o.s_hi < j ? o.s_hi : j;
        if (o.s_lo > hi) continue;
        if (hi >= last_src) {
          printf("ORDER tile (%d,%d): %s after source %d\n", k, j, desc(o).c_str(), last_src);
          return 1;
        }
        last_src = o.s_lo;
        for (int r = o.s_lo; r <= hi; ++r) {
          cover[r] += 1;
          if (solved_at[r] > a) {
            printf("EARLY %s reads source %d before it is solved\n", desc(o).c_str(), r);
            return 1;
          }
        }
        if (solved_at[k] < a) {
          printf("LATE %s updates row %d after it was solved\n", desc(o).c_str(), k);
          return 1;
        }
      }
      for (int r = k + 1; r <= j; ++r)
        if (cover[r] != 1) {
          printf("COVER term (k=%d, r=%d, j=%d) applied %d times\n", k, r, j, cover[r]);
          return 1;
        }
    }
  printf("OK %d launches %d waits\n", n, rp.nwait);
  return 0;
}
