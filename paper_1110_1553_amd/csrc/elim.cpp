// Elimination lists (Sections III and IV of the paper) and the kernel task
// graph of Algorithm 2, built on the host.
#include "elim.hpp"

#include <algorithm>
#include <cstring>
#include <queue>
#include <sstream>
#include <tuple>

namespace hqr {

// ---------------------------------------------------------------------------
// Static trees on an ascending participant list (rows[0] survives).

static void tree_flat(const std::vector<int32_t>& L, std::vector<Kill>& out) {
  // Section III-A, Table 1: one killer, top to bottom.
  for (size_t j = 1; j < L.size(); ++j) out.push_back({L[j], L[0], (int32_t)j});
}

static void tree_binary(const std::vector<int32_t>& L, std::vector<Kill>& out) {
  // Section III-A, Table 4: pairs at distance 1, 2, 4, ...
  const size_t s = L.size();
  int32_t round = 1;
  for (size_t d = 1; d < s; d <<= 1, ++round)
    for (size_t j = 0; j + d < s; j += 2 * d) out.push_back({L[j + d], L[j], round});
}

static void tree_fibonacci(const std::vector<int32_t>& L, std::vector<Kill>& out) {
  // Order-1 Fibonacci scheme: positions 1..s-1 form groups of nominal sizes
  // 1, 2, 3, ... (the last one cut short by the end of the list); the bottom
  // group dies first, and the victim at position v of group g is killed by
  // position v - g.  The killer depends on the position only, so each panel
  // repeats the previous panel's pattern one row lower.
  const int32_t s = (int32_t)L.size();
  int32_t G = 0;
  for (int32_t pos = 1, size = 1; pos < s; pos += size, ++size) ++G;
  for (int32_t pos = 1, g = 1; pos < s; pos += g, ++g) {
    const int32_t end = std::min(pos + g, s);
    for (int32_t v = pos; v < end; ++v) out.push_back({L[v], L[v - g], G - g + 1});
  }
}

static void tree_chain(const std::vector<int32_t>& L, std::vector<Kill>& out) {
  // Domino (Section IV-B): bottom row first, each killed by the row above.
  const int32_t s = (int32_t)L.size();
  for (int32_t j = s - 1; j >= 1; --j) out.push_back({L[j], L[j - 1], s - j});
}

void tree_static(int kind, const std::vector<int32_t>& rows, std::vector<Kill>& out) {
  switch (kind) {
    case HQR_FLAT: tree_flat(rows, out); break;
    case HQR_BINARY: tree_binary(rows, out); break;
    case HQR_FIBONACCI: tree_fibonacci(rows, out); break;
    case HQR_CHAIN: tree_chain(rows, out); break;
    default: break;
  }
}

// Greedy (Section III-B, Table 5): at step s, the rows of the panel that are
// alive and ready (zeroed in the previous panel before step s) are counted,
// and the bottom half of them is killed by the rows right above, pairing in
// natural order.  `ready[r]` is the step row r was zeroed at in the previous
// panel within the same (level, group), 0 if it was not.
static void tree_greedy(const std::vector<int32_t>& L, const int32_t* ready, std::vector<Kill>& out,
                        int32_t* zeroed_at) {
  std::vector<int32_t> alive(L), avail;
  avail.reserve(L.size());
  for (int32_t step = 1; alive.size() > 1; ++step) {
    avail.clear();
    for (int32_t r : alive)
      if ((ready ? ready[r] : 0) < step) avail.push_back(r);
    const size_t n = avail.size(), z = n / 2;
    if (z == 0) continue;
    for (size_t j = 0; j < z; ++j) {
      const int32_t victim = avail[n - z + j];
      out.push_back({victim, avail[n - 2 * z + j], step});
      if (zeroed_at) zeroed_at[victim] = step;
    }
    // the victims are the last z available rows; drop them from `alive`
    const int32_t first_victim = avail[n - z];
    std::vector<int32_t> keep;
    keep.reserve(alive.size());
    size_t vi = n - z;
    for (int32_t r : alive) {
      if (vi < n && r == avail[vi]) { ++vi; continue; }
      keep.push_back(r);
    }
    (void)first_victim;
    alive.swap(keep);
  }
}

int check_params(const hqr_params& p) {
  if (p.nb != 64 && p.nb != 128 && p.nb != 256) return -1;
  if (p.ib != 16) return -2;
  if (p.p < 1) return -3;
  if (p.a < 1) return -4;
  if (p.low < HQR_FLAT || p.low > HQR_FIBONACCI) return -5;
  if (p.high < HQR_FLAT || p.high > HQR_FIBONACCI) return -6;
  if (p.coupling < HQR_FLAT || p.coupling > HQR_CHAIN) return -7;
  if (p.domino != 0 && p.domino != 1) return -8;
  if (p.precision < HQR_PREC_FP64 || p.precision > HQR_PREC_BF16) return -9;
  return 0;
}

namespace {

// Greedy readiness per (level, group), kept for the previous and the current
// panel.  Levels 1..3; groups are clusters (level 3 has one group).
struct GreedyMemory {
  int32_t mt, P;
  std::vector<std::vector<int32_t>> prev, cur;
  GreedyMemory(int32_t mt_, int32_t P_) : mt(mt_), P(P_), prev(3 * P_), cur(3 * P_) {}
  void next_panel() {
    prev.swap(cur);
    for (auto& v : cur) v.clear();
  }
  void run(int kind, int level, int group, const std::vector<int32_t>& rows, std::vector<Kill>& out) {
    if (rows.size() < 2) return;
    if (kind != HQR_GREEDY) {
      tree_static(kind, rows, out);
      return;
    }
    const int slot = (level - 1) * P + group;
    std::vector<int32_t>& now = cur[slot];
    if (now.empty()) now.assign(mt, 0);
    const std::vector<int32_t>& before = prev[slot];
    tree_greedy(rows, before.empty() ? nullptr : before.data(), out, now.data());
  }
};

}  // namespace

// Hierarchical elimination list (Section IV-A/B).  Row i belongs to cluster
// i mod p with local index i / p.  For panel k and cluster c, the rows of
// the cluster at or below row k are local indices l_first..l_end-1; the top
// tile is l_first.  With the coupling level on, the local rows on or below
// the local diagonal (l >= k) are reduced by levels 0 and 1 into row l = k,
// and the coupling tree reduces [top, ..., k] into the top tile; without it
// levels 0 and 1 reduce the whole local column into the top tile.  Level 0
// kills every row of a domain of `a` local rows (aligned on multiples of a,
// cut at the first row) by the domain head with TS kernels; level 1 reduces
// the domain heads with the low tree; level 3 reduces the p top tiles with
// the high tree.
std::vector<Elim> make_elimlist(int32_t mt, int32_t nt, const hqr_params& prm) {
  std::vector<Elim> out;
  const int32_t K = std::min(mt, nt), P = prm.p, a = prm.a;
  GreedyMemory mem(mt, P);
  struct L0 { int32_t c, killer, victim, round; };
  struct LT { int32_t c, round, victim, killer; };
  std::vector<L0> lv0;
  std::vector<LT> lv1, lv2, lv3;
  std::vector<int32_t> rows, tops;
  std::vector<Kill> kills;
  for (int32_t k = 0; k < K; ++k) {
    mem.next_panel();
    lv0.clear(); lv1.clear(); lv2.clear(); lv3.clear(); tops.clear();
    for (int32_t c = 0; c < P; ++c) {
      const int32_t l_first = (k <= c) ? 0 : (k - c + P - 1) / P;
      const int32_t l_end = (mt - c + P - 1) / P;  // rows c, c+P, ... below mt
      if (l_first >= l_end) continue;
      auto glob = [&](int32_t l) { return l * P + c; };
      const int32_t top = l_first;
      tops.push_back(glob(top));
      const int32_t s0 = prm.domino ? std::max(l_first, k) : l_first;
      if (s0 < l_end) {
        for (int32_t l = s0 + 1; l < l_end; ++l) {
          const int32_t head = std::max(a * (l / a), s0);
          if (head != l) lv0.push_back({c, glob(head), glob(l), l - head});
        }
        rows.clear();
        rows.push_back(glob(s0));
        for (int32_t l = s0 + 1; l < l_end; ++l)
          if (l % a == 0) rows.push_back(glob(l));
        kills.clear();
        mem.run(prm.low, 1, c, rows, kills);
        for (const Kill& q : kills) lv1.push_back({c, q.round, q.victim, q.killer});
      }
      if (prm.domino) {
        rows.clear();
        rows.push_back(glob(top));
        for (int32_t l = top + 1; l <= k && l < l_end; ++l) rows.push_back(glob(l));
        kills.clear();
        mem.run(prm.coupling, 2, c, rows, kills);
        for (const Kill& q : kills) lv2.push_back({c, q.round, q.victim, q.killer});
      }
    }
    std::sort(tops.begin(), tops.end());
    kills.clear();
    mem.run(prm.high, 3, 0, tops, kills);
    for (const Kill& q : kills) lv3.push_back({0, q.round, q.victim, q.killer});

    std::sort(lv0.begin(), lv0.end(), [](const L0& x, const L0& y) {
      return std::tie(x.c, x.killer, x.victim) < std::tie(y.c, y.killer, y.victim);
    });
    auto by_c_round_victim = [](const LT& x, const LT& y) {
      return std::tie(x.c, x.round, x.victim) < std::tie(y.c, y.round, y.victim);
    };
    std::sort(lv1.begin(), lv1.end(), by_c_round_victim);
    std::sort(lv2.begin(), lv2.end(), by_c_round_victim);
    std::sort(lv3.begin(), lv3.end(), by_c_round_victim);
    for (const L0& e : lv0) out.push_back({k, e.victim, e.killer, HQR_KIND_TS, 0, e.round});
    for (const LT& e : lv1) out.push_back({k, e.victim, e.killer, HQR_KIND_TT, 1, e.round});
    for (const LT& e : lv2) out.push_back({k, e.victim, e.killer, HQR_KIND_TT, 2, e.round});
    for (const LT& e : lv3) out.push_back({k, e.victim, e.killer, HQR_KIND_TT, 3, e.round});
  }
  return out;
}

// Validity rules of Section II.  `zeroed[r]` counts the panels in which row r
// has been killed so far; rows are killed panel after panel, so row r is
// ready for panel k -- and, for a killer, still alive in it -- exactly when
// zeroed[r] == k.
std::string validate_elimlist(int32_t mt, int32_t nt, const Elim* list, int64_t count) {
  std::ostringstream why;
  const int32_t K = std::min(mt, nt);
  std::vector<int32_t> zeroed(mt, 0);
  std::vector<uint8_t> ts_victim((size_t)mt * K, 0);
  for (int64_t n = 0; n < count; ++n) {
    const Elim& e = list[n];
    if (e.k < 0 || e.k >= K || e.victim <= e.k || e.victim >= mt || e.killer < e.k || e.killer >= mt ||
        e.killer == e.victim || (e.kind != HQR_KIND_TS && e.kind != HQR_KIND_TT)) {
      why << "record " << n << " out of range";
      return why.str();
    }
    if (zeroed[e.victim] != e.k) {
      why << "record " << n << ": row " << e.victim << " is not ready for panel " << e.k
          << " or is already zero";
      return why.str();
    }
    if (zeroed[e.killer] != e.k) {
      why << "record " << n << ": killer " << e.killer << " is not ready for panel " << e.k
          << " or is already zero";
      return why.str();
    }
    zeroed[e.victim] = e.k + 1;
    if (e.kind == HQR_KIND_TS) ts_victim[(size_t)e.victim * K + e.k] = 1;
  }
  for (int32_t r = 0; r < mt; ++r)
    if (zeroed[r] != std::min(r, K)) {
      why << "row " << r << " zeroed in " << zeroed[r] << " panels, expected " << std::min(r, K);
      return why.str();
    }
  for (int64_t n = 0; n < count; ++n)
    if (ts_victim[(size_t)list[n].killer * K + list[n].k]) {
      why << "record " << n << ": TS victim " << list[n].killer << " used as a killer";
      return why.str();
    }
  return std::string();
}

std::vector<Task> expand_tasks(int32_t mt, int32_t nt, const std::vector<Elim>& list, int32_t ncols) {
  if (ncols < nt) ncols = nt;
  std::vector<Task> tasks;
  const int32_t K = std::min(mt, nt);
  std::vector<uint8_t> ts_victim(mt);
  size_t n = 0;
  for (int32_t k = 0; k < K; ++k) {
    size_t end = n;
    while (end < list.size() && list[end].k == k) ++end;
    std::fill(ts_victim.begin(), ts_victim.end(), 0);
    for (size_t q = n; q < end; ++q)
      if (list[q].kind == HQR_KIND_TS) ts_victim[list[q].victim] = 1;
    for (int32_t r = k; r < mt; ++r) {
      if (ts_victim[r]) continue;
      tasks.push_back({GEQRT, r, -1, k, -1});
      for (int32_t j = k + 1; j < ncols; ++j) tasks.push_back({UNMQR, r, -1, k, j});
    }
    for (size_t q = n; q < end; ++q) {
      const Elim& e = list[q];
      const bool ts = e.kind == HQR_KIND_TS;
      tasks.push_back({(uint8_t)(ts ? TSQRT : TTQRT), e.victim, e.killer, k, -1});
      for (int32_t j = k + 1; j < ncols; ++j) tasks.push_back({(uint8_t)(ts ? TSMQR : TTMQR), e.victim, e.killer, k, j});
    }
    n = end;
  }
  return tasks;
}

// Device plan: split every update into `chunks` column chunks, give each
// task the dependency-counter versions it must wait for, and order the tasks
// for dispatch.
//
// Dependency model.  Each tile has one write counter per column chunk.  A
// panel task (GEQRT/TSQRT/TTQRT) writes every chunk of its tiles; an update
// chunk writes one chunk of its two (or one) tiles.  Tiles read but not
// written -- the Householder vectors and T of a finished panel task -- are
// never written again, so reads need no ordering against later writes.  A
// task therefore waits until every counter it touches has reached the number
// of earlier writes in program order, and bumps the counters it writes when
// done.
int build_plan(int32_t mt, int32_t nt, const hqr_params& prm, int order, int chunks, Plan& plan,
               const ColumnChunks& ccfg) {
  plan = Plan();
  plan.mt = mt;
  plan.nt = nt;
  plan.nb = prm.nb;
  plan.chunks = chunks;
  plan.list = make_elimlist(mt, nt, prm);
  {
    std::string why = validate_elimlist(mt, nt, plan.list.data(), (int64_t)plan.list.size());
    if (!why.empty()) return HQR_ERR_INTERNAL;
  }
  // tile columns of the launch and their active chunks
  const int32_t nrt = (ccfg.nrhs_cols + prm.nb - 1) / prm.nb;  // right-hand-side tile columns
  const int32_t ncols = nt + nrt;
  std::vector<int32_t> active(ncols, chunks);
  if (ccfg.last_a > 0 && ccfg.last_a < chunks) active[nt - 1] = ccfg.last_a;
  const int32_t cw = prm.nb / chunks;      // columns per counter sub-chunk
  const int S = (prm.nb >= 128) ? 2 : 1;  // sub-chunks per update task (128 columns)
  if (nrt > 0) active[ncols - 1] = ((ccfg.nrhs_cols - (nrt - 1) * prm.nb) + cw - 1) / cw;
  const std::vector<Task> tasks = expand_tasks(mt, nt, plan.list, ncols);
  hqr_dag_info& info = plan.info;
  info.eliminations = (int64_t)plan.list.size();
  info.tasks = (int64_t)tasks.size();
  for (const Task& t : tasks) {
    info.count[t.op]++;
    info.weight += op_weight(t.op);
  }

  const size_t ntiles = (size_t)mt * ncols;
  std::vector<uint32_t> writes(ntiles, 0);
  std::vector<int64_t> last_writer(ntiles * chunks, -1);
  std::vector<DevTask> dev;
  std::vector<int64_t> wt;  // integer weight of each device task, units of b^3/(3 chunks)
  std::vector<int64_t> pred_off{0}, preds;
  dev.reserve(tasks.size() * chunks);
  auto tile = [&](int32_t r, int32_t c) { return (size_t)r * ncols + c; };
  auto add_pred = [&](int64_t p) {
    if (p < 0) return;
    for (int64_t q = pred_off.back(); q < (int64_t)preds.size(); ++q)
      if (preds[q] == p) return;
    preds.push_back(p);
  };
  for (const Task& t : tasks) {
    const bool panel = (t.op == GEQRT || t.op == TSQRT || t.op == TTQRT);
    if (panel) {
      DevTask d{};
      d.op = t.op;
      d.k = (uint16_t)t.k;
      d.j = (uint16_t)t.k;
      const int ca = active[t.k];
      d.chunk = (uint8_t)ca;
      const int64_t id = (int64_t)dev.size();
      if (t.op == GEQRT) {
        d.row = d.killer = (uint16_t)t.row;
        const size_t x = tile(t.row, t.k);
        d.v[0] = writes[x];
        for (int c = 0; c < ca; ++c) add_pred(last_writer[x * chunks + c]);
        writes[x]++;
        for (int c = 0; c < ca; ++c) last_writer[x * chunks + c] = id;
      } else {
        d.row = (uint16_t)t.row;
        d.killer = (uint16_t)t.killer;
        const size_t xp = tile(t.killer, t.k), xi = tile(t.row, t.k);
        d.v[0] = writes[xp];
        d.v[1] = writes[xi];
        for (int c = 0; c < ca; ++c) {
          add_pred(last_writer[xp * chunks + c]);
          add_pred(last_writer[xi * chunks + c]);
        }
        writes[xp]++;
        writes[xi]++;
        for (int c = 0; c < ca; ++c) last_writer[xp * chunks + c] = last_writer[xi * chunks + c] = id;
      }
      dev.push_back(d);
      wt.push_back((int64_t)op_weight(t.op) * chunks);
      pred_off.push_back((int64_t)preds.size());
    } else {
      // update: read tile (row,k) [UNMQR] or (victim,k) [TS/TT]; write (killer,j) and (row,j)
      const size_t xv = tile(t.row, t.k), xi = tile(t.row, t.j);
      const size_t xp = (t.op == UNMQR) ? 0 : tile(t.killer, t.j);
      // one device task per S sub-chunks of column j (only those that hold
      // matrix columns); it waits for the factored tile's last active
      // sub-chunk, which its panel task publishes when done
      const int cv = active[t.k] - 1;
      const int nu = (active[t.j] + S - 1) / S;
      for (int u = 0; u < nu; ++u) {
        const int c0 = u * S, cn = std::min(S, active[t.j] - c0);
        DevTask d{};
        d.op = t.op;
        d.chunk = (uint8_t)c0;
        d.pad = (uint16_t)(cv | (cn << 8));
        d.row = (uint16_t)t.row;
        d.killer = (uint16_t)(t.op == UNMQR ? t.row : t.killer);
        d.k = (uint16_t)t.k;
        d.j = (uint16_t)t.j;
        d.v[0] = writes[xv];
        add_pred(last_writer[xv * chunks + cv]);
        if (t.op == UNMQR) {
          d.v[1] = writes[xi];
        } else {
          d.v[1] = writes[xp];
          d.v[2] = writes[xi];
        }
        for (int c = c0; c < c0 + cn; ++c) {
          if (t.op != UNMQR) add_pred(last_writer[xp * chunks + c]);
          add_pred(last_writer[xi * chunks + c]);
        }
        const int64_t id = (int64_t)dev.size();
        for (int c = c0; c < c0 + cn; ++c) {
          if (t.op != UNMQR) last_writer[xp * chunks + c] = id;
          last_writer[xi * chunks + c] = id;
        }
        dev.push_back(d);
        wt.push_back((int64_t)op_weight(t.op) * cn);
        pred_off.push_back((int64_t)preds.size());
      }
      if (t.op != UNMQR) writes[xp]++;
      writes[xi]++;
    }
  }
  const int64_t nd = (int64_t)dev.size();
  info.device_tasks = nd;

  // successors (CSR) and bottom levels: edges always point forward in program
  // order, so a reverse sweep sees every successor before its predecessors.
  std::vector<int64_t> nsucc(nd + 1, 0);
  for (int64_t q = 0; q < (int64_t)preds.size(); ++q) nsucc[preds[q] + 1]++;
  for (int64_t i = 0; i < nd; ++i) nsucc[i + 1] += nsucc[i];
  std::vector<int64_t> succ(preds.size()), fill(nsucc.begin(), nsucc.end() - 1);
  for (int64_t i = 0; i < nd; ++i)
    for (int64_t q = pred_off[i]; q < pred_off[i + 1]; ++q) succ[fill[preds[q]]++] = i;
  std::vector<int64_t> bottom(nd, 0), prio(nd, 0);
  int64_t cp = 0;
  for (int64_t i = nd - 1; i >= 0; --i) {
    int64_t best = 0, bestp = 0;
    for (int64_t q = nsucc[i]; q < nsucc[i + 1]; ++q) {
      best = std::max(best, bottom[succ[q]]);
      bestp = std::max(bestp, prio[succ[q]]);
    }
    bottom[i] = wt[i] + best;
    // dispatch priority: panel kernels run far below their flop rate, so they
    // count three times their weight on the path
    const bool panel = dev[i].op == GEQRT || dev[i].op == TSQRT || dev[i].op == TTQRT;
    prio[i] = wt[i] * (panel ? 3 : 1) + bestp;
    cp = std::max(cp, bottom[i]);
  }
  info.critical_path = (cp + chunks - 1) / chunks;

  if (order == 1) {
    plan.dev.swap(dev);
    plan.prio.swap(prio);
    return 0;
  }
  // Dispatch order: a list schedule simulated on kSimWorkers workers with
  // estimated task durations.  A task becomes ready when its predecessors
  // have finished in simulated time, and a free worker takes the ready task
  // with the longest remaining path (in the same time estimate).  Listing
  // tasks in this order keeps workgroups from taking tasks whose inputs are
  // far from ready (a plain topological order by path length lists whole
  // dependency chains back to back, and the workgroups that take them wait on
  // each other).  Durations (microseconds at nb = 256, from measurements of
  // the tile kernels): panel tasks are latency bound (~470 us for a full
  // tile, proportional to nb), update tasks scale with their flops, plus a
  // fixed per-task cost.  A panel task publishes its tile block by block, so
  // the panel tasks that depend on it can start one block after it starts;
  // every other successor waits for its end.
  constexpr int kSimWorkers = 256;
  const double s = prm.nb / 256.0;
  std::vector<double> dur(nd), bl(nd, 0.0);
  for (int64_t i = 0; i < nd; ++i) {
    const int op = dev[i].op;
    if (op == GEQRT || op == TSQRT || op == TTQRT) {
      dur[i] = 470.0 * s * (double)dev[i].chunk / chunks + 10.0;
    } else {
      const double per_unit = (op == TSMQR) ? 6.5 : 8.7;  // TSMQR runs closest to the MFMA rate
      dur[i] = per_unit * (double)wt[i] * s * s * s + 8.0;
    }
  }
  auto is_panel = [&](int64_t i) { return dev[i].op == GEQRT || dev[i].op == TSQRT || dev[i].op == TTQRT; };
  std::vector<double> lead(nd);  // time after its start at which a panel task's panel successors may start
  for (int64_t i = 0; i < nd; ++i) lead[i] = is_panel(i) ? dur[i] / std::max<int>(1, dev[i].chunk) : dur[i];
  for (int64_t i = nd - 1; i >= 0; --i) {
    double best = dur[i];
    for (int64_t q = nsucc[i]; q < nsucc[i + 1]; ++q) {
      const int64_t j = succ[q];
      best = std::max(best, (is_panel(i) && is_panel(j) ? lead[i] : dur[i]) + bl[j]);
    }
    bl[i] = best;
  }
  std::vector<int32_t> indeg(nd, 0);
  for (int64_t i = 0; i < nd; ++i) indeg[i] = (int32_t)(pred_off[i + 1] - pred_off[i]);
  typedef std::pair<double, int64_t> Key;  // (remaining path, -index)
  std::priority_queue<Key> ready;
  // events: (time, task, kind) with kind 0 = the first block of a panel task
  // is published (its panel successors), 1 = the task ends
  typedef std::tuple<double, int64_t, int> Event;
  std::priority_queue<Event, std::vector<Event>, std::greater<Event>> running;
  for (int64_t i = 0; i < nd; ++i)
    if (indeg[i] == 0) ready.push({bl[i], -i});
  plan.dev.reserve(nd);
  plan.prio.reserve(nd);
  int free_workers = kSimWorkers;
  double now = 0.0;
  while ((int64_t)plan.dev.size() < nd) {
    while (free_workers > 0 && !ready.empty()) {
      const int64_t i = -ready.top().second;
      ready.pop();
      plan.dev.push_back(dev[i]);
      plan.prio.push_back((int64_t)(bl[i] * 16.0));
      if (is_panel(i)) running.push(Event{now + lead[i], i, 0});
      running.push(Event{now + dur[i], i, 1});
      --free_workers;
    }
    if ((int64_t)plan.dev.size() == nd) break;
    if (running.empty()) return HQR_ERR_INTERNAL;  // a dependency cycle (cannot happen: edges point forward)
    now = std::get<0>(running.top());
    while (!running.empty() && std::get<0>(running.top()) <= now) {
      const int64_t j = std::get<1>(running.top());
      const int kind = std::get<2>(running.top());
      running.pop();
      if (kind == 1) ++free_workers;
      for (int64_t q = nsucc[j]; q < nsucc[j + 1]; ++q) {
        const int64_t sq = succ[q];
        // panel -> panel edges are released by the first-block event, the others at the end
        const bool early = is_panel(j) && is_panel(sq);
        if (early != (kind == 0)) continue;
        if (--indeg[sq] == 0) ready.push({bl[sq], -sq});
      }
    }
  }
  return 0;
}

int build_apply_plan(int32_t mt, int32_t nt, int32_t nbc, const hqr_params& prm, int trans, Plan& plan) {
  plan = Plan();
  plan.mt = mt;
  plan.nt = nt;
  plan.nb = prm.nb;
  plan.chunks = 1;
  plan.list = make_elimlist(mt, nt, prm);
  if (!validate_elimlist(mt, nt, plan.list.data(), (int64_t)plan.list.size()).empty()) return HQR_ERR_INTERNAL;
  // the transformations that act on B: one per triangularisation (GEQRT ->
  // UNMQR) and one per elimination (TSQRT -> TSMQR, TTQRT -> TTMQR)
  std::vector<Task> ops;
  for (const Task& t : expand_tasks(mt, std::max(nt, 1), plan.list)) {
    if (t.op == GEQRT) ops.push_back({UNMQR, t.row, -1, t.k, -1});
    if (t.op == TSQRT) ops.push_back({TSMQR, t.row, t.killer, t.k, -1});
    if (t.op == TTQRT) ops.push_back({TTMQR, t.row, t.killer, t.k, -1});
  }
  if (!trans) std::reverse(ops.begin(), ops.end());
  std::vector<uint32_t> writes((size_t)mt * nbc, 0);
  plan.dev.reserve(ops.size() * nbc);
  for (const Task& t : ops) {
    for (int32_t b = 0; b < nbc; ++b) {
      DevTask d{};
      d.op = t.op;
      d.chunk = 0;
      d.row = (uint16_t)t.row;
      d.killer = (uint16_t)(t.op == UNMQR ? t.row : t.killer);
      d.k = (uint16_t)t.k;
      d.j = (uint16_t)b;
      d.v[0] = 0;
      const size_t xi = (size_t)t.row * nbc + b;
      if (t.op == UNMQR) {
        d.v[1] = writes[xi];
      } else {
        const size_t xp = (size_t)t.killer * nbc + b;
        d.v[1] = writes[xp];
        d.v[2] = writes[xi];
        writes[xp]++;
      }
      writes[xi]++;
      plan.dev.push_back(d);
      plan.info.count[t.op]++;
      plan.info.weight += op_weight(t.op);
    }
  }
  plan.info.eliminations = (int64_t)plan.list.size();
  plan.info.tasks = plan.info.device_tasks = (int64_t)plan.dev.size();
  return 0;
}

}  // namespace hqr
