// Host-side plan of the iteration launches of a time step whose queued
// launches left it undecided (pure integer arithmetic, no HIP: the CPU tests
// compile this header on its own).
//
// A step resumed from the host gets batches of iteration launches, each
// followed by an end of step that judges the batch's iterates: the extra-th
// batch has resume_count(extra) launches (1, 1, 2, 4, ... up to kMaxBatch),
// cut to the iteration limit and to what one ring of iterate buffers holds.
#pragma once

namespace ocip {

constexpr int kMaxBatch = 64;   // iteration launches per batch at most

// Launches of the extra-th batch after a step's first (extra >= 1).  The
// shift is bounded: a slow step can need thousands of batches.
inline int resume_count(int extra) {
  if (extra <= 2) return 1;
  if (extra - 2 >= 30) return kMaxBatch;
  const int n = 1 << (extra - 2);
  return n < kMaxBatch ? n : kMaxBatch;
}

// The extra-th resumed batch of a step that has `launched` iterates so far:
// resume_count(extra), at most max_iters - launched (but at least one: the
// end of step then stops at the iteration limit) and at most nbuf - 1 (the
// end of step reads the records of one ring of nbuf slots).
inline int resumed_batch(int extra, int launched, int max_iters, int nbuf) {
  int n = resume_count(extra);
  const int left = max_iters - launched > 1 ? max_iters - launched : 1;
  if (n > left) n = left;
  if (n > nbuf - 1) n = nbuf - 1;
  return n;
}

// A batch of `count` single-iterate launches after iterate cb.
inline bool batch_range_ok(int cb, int count) {
  return cb >= 0 && count >= 1 && count <= kMaxBatch;
}

// An end of step over iterates first .. last, whose records sit in a ring of
// nbuf slots (iterate l in slot l % nbuf; the end also reads iterate first-1).
inline bool end_range_ok(int first, int last, int nbuf) {
  return first >= 1 && last >= first && last - first < nbuf - 1;
}

// Ensemble launches of up to ki iterates each (ki = 1, 3 or 4) over a batch
// whose problems plan different iterate ranges first .. last: a class of
// problems launches at nodes 1, 1 + ki, 1 + 2 ki, ... up to its longest
// range.  (constexpr: the queue kernels evaluate the same functions.)
constexpr bool ens_launch_node(int node, int ki) { return node >= 1 && (node - 1) % ki == 0; }

// Iterates that the launch at `node` computes for a problem planning
// first .. last: iterates first + node - 1 onwards, at most ki, none past
// last (0: the problem's work-groups are idle).
constexpr int ens_levels(int first, int last, int node, int ki) {
  const int n = last - (first - 1 + node) + 1;
  return n < 0 ? 0 : (n < ki ? n : ki);
}

// Iterates that the launch's reduction work-group reduces: those of the
// problem's launch before (ki of them; none at node 1, where the iterates
// before first were reduced with the batch before).
constexpr int ens_reduced_before(int node, int ki) {
  return node - 1 < ki ? node - 1 : ki;
}

// Iterates of the problem's last launch, which the batch's final reduction
// reduces: last - ki + 1 .. last for a full launch, fewer for a partial one.
constexpr int ens_trailing(int first, int last, int ki) { return (last - first) % ki + 1; }

}  // namespace ocip
