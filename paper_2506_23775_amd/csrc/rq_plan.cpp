// Sweep-pass scheduler.
//
// The paper applies gates one at a time, each reading and writing the whole
// state (Sec. "Gate application"; Sec. "Parallelization": the kernels are
// memory bound).  Gates on disjoint qubits commute, so any reordering that
// keeps the order of gates sharing a qubit gives the same circuit (the
// paper's sequentialisation of a brick wall, Sec. "Brick wall circuit
// layout", is one such order).  The scheduler exploits this to apply several
// gates per pass over the state: a pass owns a tile of `nt` explicit qubits
// and takes, in circuit order, every not yet applied gate that lies inside the
// tile and is not preceded by a skipped gate on one of its qubits.
//
// Tile choice (greedy, deterministic): for every gate on the current
// frontier, start from its qubits and repeatedly add the qubits of the
// blocked-by-tile gate that needs the fewest new qubits (ties: lowest gate
// index) while the tile has room; keep the seed whose tile takes the most
// gates (ties: lowest seed index).
#include "rq_plan.h"

#include <algorithm>

namespace rqk {

namespace {

struct Closure {
  std::vector<int> taken;
  std::vector<int> cands;
};

}  // namespace

bool plan_passes(int k, int n, const int32_t *pairs, bool parity, int nt, int maxg,
                 std::vector<PlanPass> &out, std::string &err) {
  out.clear();
  const int kq = parity ? k - 1 : k;
  if (nt < 2 || nt > 8 || nt > kq) {
    err = "tile size out of range";
    return false;
  }
  std::vector<uint32_t> qm(n), em(n);
  for (int g = 0; g < n; ++g) {
    const int a = pairs[2 * g], b = pairs[2 * g + 1];
    if (a < 0 || b < 0 || a >= k || b >= k || a == b) {
      err = "gate " + std::to_string(g) + ": invalid qubit pair";
      return false;
    }
    qm[g] = (1u << a) | (1u << b);
    em[g] = qm[g];
    if (parity) em[g] &= ~(1u << (k - 1));
  }
  std::vector<char> done(n, 0);
  int remaining = n;

  auto closure = [&](uint32_t Q) {
    Closure c;
    uint32_t blocked = 0;
    for (int g = 0; g < n; ++g) {
      if (done[g]) continue;
      if (blocked & qm[g]) {
        blocked |= qm[g];
        continue;
      }
      const bool fits = (em[g] & ~Q) == 0;
      if (fits && (int)c.taken.size() < maxg) {
        c.taken.push_back(g);
      } else {
        if (!fits) c.cands.push_back(g);
        blocked |= qm[g];
      }
    }
    return c;
  };

  while (remaining > 0) {
    std::vector<int> frontier;
    {
      uint32_t blocked = 0;
      for (int g = 0; g < n; ++g) {
        if (done[g]) continue;
        if (!(blocked & qm[g])) frontier.push_back(g);
        blocked |= qm[g];
      }
    }
    int best_score = -1;
    uint32_t best_Q = 0;
    for (int seed : frontier) {
      uint32_t Q = em[seed];
      for (;;) {
        Closure c = closure(Q);
        int pick = -1, pick_new = 1 << 30;
        for (int g : c.cands) {
          const uint32_t add = em[g] & ~Q;
          const int nn = __builtin_popcount(add);
          if (__builtin_popcount(Q | em[g]) > nt) continue;
          if (nn < pick_new) {
            pick_new = nn;
            pick = g;
          }
        }
        if (pick < 0 || (int)c.taken.size() >= maxg) break;
        Q |= em[pick];
      }
      const int score = (int)closure(Q).taken.size();
      if (score > best_score) {
        best_score = score;
        best_Q = Q;
      }
    }
    Closure c = closure(best_Q);
    if (c.taken.empty()) {
      err = "scheduler made no progress";
      return false;
    }
    // pad the tile to exactly nt explicit qubits
    uint32_t Q = best_Q;
    for (int q = 0; q < kq && __builtin_popcount(Q) < nt; ++q) Q |= 1u << q;
    PlanPass pp;
    int local[32];
    int b = 0;
    for (int q = 0; q < kq; ++q) {
      local[q] = -1;
      if ((Q >> q) & 1) {
        local[q] = b;
        pp.pos[b] = kq - 1 - q;
        pp.qmask |= 1u << (kq - 1 - q);
        ++b;
      }
    }
    for (int g : c.taken) {
      GateRef r;
      r.inst = (int16_t)g;
      const int qh = pairs[2 * g], ql = pairs[2 * g + 1];
      if (parity && ql == k - 1) {
        r.kind = 1;
        r.h = (int16_t)local[qh];
        r.l = 0;
      } else if (parity && qh == k - 1) {
        r.kind = 2;
        r.h = (int16_t)local[ql];
        r.l = 0;
      } else {
        r.kind = 0;
        r.h = (int16_t)local[qh];
        r.l = (int16_t)local[ql];
      }
      pp.gates.push_back(r);
      done[g] = 1;
      --remaining;
    }
    out.push_back(pp);
  }
  return true;
}

}  // namespace rqk
