// Band wavefront schedule of Algorithm 1 (Section 3) for one pencil: the order in
// which the tile solves and tile updates are enqueued on two streams, with the events
// that order them.  Host code only, no HIP types: the operations are supplied by the
// caller (Ops), so the same schedule drives the HIP launches and the host-side replay
// that checks its ordering.
//
// Tile rows [0, rows) are grouped into bands of R rows, band b = rows [R b, R b + R - 1].
// For each band from the bottom:
//   C(b)   on the caller's stream A: the band's rows from the bottom up, each solve
//          followed by the small update of the band rows above it (one launch per step, or
//          one launch for all of them: ops.chain);
//   U1(b)  on A: the band applied to the next band's rows [R (b - 1), R b);
//   U2(b)  on the side stream B: the band applied to every row above, [0, R (b - 1)), in
//          launches of about `split` tiles each (whole tile rows, from the bottom; 0: one
//          launch).  The launches are independent; their boundaries give the chain's
//          launches on A a share of the GPU, which a single large launch keeps to itself
//          until its last workgroups are placed.
// Dependencies (every one is an event or stream order):
//   U1(b)  needs U2(b + 1), which also read-modifies-writes rows of band b - 1 (the
//          sources of a tile are applied in descending order, and a tile column's first
//          update overwrites rather than accumulates), so the two must not overlap;
//   C(b)   needs U2(b + 2), the last writer of its rows and the last reader of the W
//          slots (two bands of them) it is about to overwrite: C(b) follows U1(b + 1)
//          on A, which waited for U2(b + 2);
//   U2(b)  needs C(b) (its sources), and stream order on B puts it after U2(b + 1); it also
//          waits for U1(b), which the chain C(b - 1) waits for: started together, the large
//          U2(b) would take the GPU from the small U1(b) and delay the chain by its length.
// C(b - 1) needs U1(b) and U2(b + 1) only, so it overlaps U2(b) (the look-ahead).
#pragma once

namespace rgev {

enum SchedStream { kStreamA = 0, kStreamB = 1 };
enum SchedEvent { kEvC = 0, kEvJ = 1, kEvU0 = 2, kEvU1 = 3 };

// Ops:  solve(i, stream)                              solve tile row i (all columns j >= i)
//       update(k_lo, k_hi, j_lo, s_lo, s_hi, stream)  sources [s_lo, s_hi] -> rows [k_lo, k_hi)
//       chain(r_lo, r_hi, stream)                     C(b): rows r_hi .. r_lo, each solve(i)
//                                                     followed by update(r_lo, i, i, i, i) (as
//                                                     these launches, or fused in one launch)
//       record(event, stream), wait(stream, event)    event order between the streams
// Each returns false on failure, which stops the enqueue.

// C(b) as separate launches, for the Ops that have no fused form
template <class Ops>
bool chain_steps(int r_lo, int r_hi, int stream, Ops& ops) {
  bool ok = true;
  for (int i = r_hi; i >= r_lo && ok; --i) {
    ok = ops.solve(i, stream);
    if (i > r_lo && ok) ok = ops.update(r_lo, i, i, i, i, stream);
  }
  return ok;
}
template <class Ops>
bool band_schedule(int rows, int R, int split, Ops& ops) {
  bool ok = true;
  auto chk = [&](bool b) { ok = ok && b; };
  // the side stream starts after everything already queued on the caller's stream
  chk(ops.record(kEvC, kStreamA));
  chk(ops.wait(kStreamB, kEvC));
  chk(ops.record(kEvU0, kStreamB));
  chk(ops.record(kEvU1, kStreamB));
  for (int b = (rows - 1) / R; b >= 0 && ok; --b) {
    const int r_lo = R * b, r_hi = R * b + R - 1;
    chk(ops.chain(r_lo, r_hi < rows ? r_hi : rows - 1, kStreamA));
    if (r_lo > 0 && ok) {
      const int nlo = r_lo > R ? r_lo - R : 0;
      // U2(b + 1): evU[(b + 1) & 1] was last recorded after it
      chk(ops.wait(kStreamA, ((b + 1) & 1) ? kEvU1 : kEvU0));
      chk(ops.update(nlo, r_lo, r_lo, r_lo, r_hi, kStreamA));
      chk(ops.record(kEvC, kStreamA));   // C(b) and U1(b)
      if (nlo > 0) {
        chk(ops.wait(kStreamB, kEvC));
        const int ncol = rows - r_lo;   // tile columns r_lo .. rows - 1
        int cr = split > 0 ? (split + ncol - 1) / ncol : nlo;   // tile rows per launch
        if (cr < 1) cr = 1;
        for (int hi = nlo; hi > 0 && ok; hi -= cr) chk(ops.update(hi - cr > 0 ? hi - cr : 0, hi, r_lo, r_lo, r_hi, kStreamB));
        chk(ops.record((b & 1) ? kEvU1 : kEvU0, kStreamB));
      }
    }
  }
  // join the side stream back into the caller's stream
  chk(ops.record(kEvJ, kStreamB));
  chk(ops.wait(kStreamA, kEvJ));
  return ok;
}

// The same schedule in lock-step over a batch of pencils: every launch is one part of step
// t for all pencils of a group, pencil p being in its band b_p = B_p - 1 - t (B_p bands of
// R tile rows from the top; a step beyond a pencil's bands is a no-op for it).  In pencil
// p's rows, r_lo = R b_p and r_hi = min(r_lo + R - 1, M_p - 1):
//   solve(t, io, s)            solves row r_hi - io (when it is >= r_lo);
//   inband(t, io, s)           source row r_hi - io applied to rows [r_lo, r_hi - io);
//   next(t, s)                 U1: the band applied to the next band's rows [r_lo - R, r_lo);
//   above(t, off, cnt, s)      part of U2: the band applied to rows [max(0, hi - cnt), hi),
//                              hi = r_lo - R - off (rows counted from the bottom).
// Each pencil sees exactly the launches and dependencies band_schedule gives it (with U2 of
// step t in launches of cr[t] rows, or one launch for cr[t] <= 0), so the look-ahead is the
// same: step t + 1's chain overlaps U2 of step t.  steps is the largest B_p; above[t]
// (t < steps) the largest U2 row count r_lo - R of step t over the group (0: no U2 launch).
template <class Ops>
bool batch_band_schedule(int steps, int R, const int* cr, const int* above, Ops& ops) {
  bool ok = true;
  auto chk = [&](bool b) { ok = ok && b; };
  chk(ops.record(kEvC, kStreamA));
  chk(ops.wait(kStreamB, kEvC));
  chk(ops.record(kEvU0, kStreamB));
  chk(ops.record(kEvU1, kStreamB));
  for (int t = 0; t < steps && ok; ++t) {
    for (int io = 0; io < R && ok; ++io) {
      chk(ops.solve(t, io, kStreamA));
      if (io + 1 < R) chk(ops.inband(t, io, kStreamA));
    }
    if (t + 1 < steps && ok) {
      // U2 of step t - 1 (evU[(t - 1) & 1] was last recorded after it)
      chk(ops.wait(kStreamA, ((t + 1) & 1) ? kEvU1 : kEvU0));
      chk(ops.next(t, kStreamA));
      chk(ops.record(kEvC, kStreamA));
      const int rows = above[t];
      if (rows > 0 && ok) {
        chk(ops.wait(kStreamB, kEvC));
        const int c = cr[t] > 0 ? cr[t] : rows;
        for (int off = 0; off < rows && ok; off += c) chk(ops.above(t, off, c, kStreamB));
        chk(ops.record((t & 1) ? kEvU1 : kEvU0, kStreamB));
      }
    }
  }
  chk(ops.record(kEvJ, kStreamB));
  chk(ops.wait(kStreamA, kEvJ));
  return ok;
}

}  // namespace rgev
