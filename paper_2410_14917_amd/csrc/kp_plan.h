// Host-side planner of the batched call: which workgroups solve which problems.
//
// The persistent batched kernel splits its grid into teams of consecutive
// workgroups.  A team solves its problems one after another, each with the
// single-problem machinery (row ownership inside the team, one team-wide
// barrier per phase, the team's first workgroup as leader).  The plan fixes
// the team sizes and which class of teams (teams of one size) each problem
// goes to; on the device the teams of a class take their class's problems,
// heaviest first, as they become free.
//
// Cost model of one problem on a team of g workgroups (seconds):
//   steps    S  = max(16, 8 sqrt(h rho)) for h rho < 64 (one substep, m
//               grown by doubling), 9.5 sqrt(h rho) above (substeps of
//               m_max = 48), rho = a Gershgorin bound of ||A||: least-squares
//               fits of the measured step counts of 512 advection-diffusion-
//               reaction problems at tol 1e-8 (h rho from 0.4 to 1e4); the
//               controller takes O(sqrt(h rho)) steps on these
//               diffusion-dominated spectra
//   m_eff       = min(S, m_max) (Krylov dimension of a substep)
//   passes   P  = S (m_eff + p + c + 6) vectors of N float64 (the per-step
//               traffic 2j + p + c + 5 averaged over a substep, plus combine)
//   time        = 8 P max(N / g, e_min) / bw_wg              (streaming)
//               + S (t_step + [g > 1] t_team + log2(g) t_log) (serial per step)
//               + (S / m_eff + r) t_expm(m_eff)              (small exponentials)
// bw_wg is one workgroup's share of HBM bandwidth with the whole grid
// streaming, e_min the element count below which a workgroup's passes are
// latency-bound.
//
// Search (the autotuner): team-size mixes  k_big teams of g_big, k_mid teams
// of g_mid, the rest single workgroups; for each mix the problems, heaviest
// first, go to the team that would finish them earliest (LPT list
// scheduling); the mix with the smallest predicted makespan wins.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <queue>
#include <vector>

namespace kp {

struct PlanProblem {
  int64_t n;       // unknowns
  int nx, ny;      // grid (rows are distributed over a team)
  int p, c;        // phi terms beyond b_0, coefficient fields read per matvec
  int m_max;
  double h_rho;    // h times a bound of ||A||
};

struct PlanModel {
  double bw_wg = 19.5e9;     // bytes/s per workgroup, whole grid streaming
  double e_min = 4096.0;     // elements per workgroup below which passes are latency-bound
  double t_step = 5.0e-6;    // serial work + pass latencies per Arnoldi step
  double t_team = 4.0e-6;    // team barriers per step (g > 1)
  double t_log = 0.5e-6;     // per doubling of the team (reductions, waits)
  double t_expm64 = 2.6e-4;  // small exponential at m = 64 (scales with m^2)
  int rejects = 4;           // rejected trials per problem (extra exponentials)
};

struct Plan {
  std::vector<int> team_size;    // workgroups of team t
  std::vector<int> team_wg0;     // first workgroup of team t
  std::vector<int> team_first;   // problems of team t: order[team_first[t] .. team_first[t+1])
  std::vector<int> order;        // problem indices grouped by team, heaviest first
  std::vector<int> team_of_wg;   // team of each workgroup of the grid (-1: idle)
  double makespan = 0.0;         // predicted seconds
  double work = 0.0;             // predicted seconds on one workgroup, all problems
  int g_big = 1, k_big = 0, g_mid = 1, k_mid = 0;
};

inline double plan_steps(const PlanProblem& q) {
  const double r = std::sqrt(std::max(0.0, q.h_rho));
  return q.h_rho < 64.0 ? std::max(16.0, 8.0 * r) : 9.5 * r;
}

// Row geometry of a problem on a team of g workgroups: rows per workgroup
// (even when nx is odd, so that every owned segment starts on an element
// pair) and the number of workgroups that own rows (<= g).
inline void plan_rows(int nx, int ny, int g, int* rows, int* nwg_rows) {
  int r = (ny + g - 1) / g;
  r = std::max(1, std::min(r, ny));
  if ((nx & 1) && (r & 1) && r < ny) ++r;
  *rows = r;
  *nwg_rows = (ny + r - 1) / r;
}

inline double plan_time(const PlanProblem& q, int g, const PlanModel& md) {
  const double S = plan_steps(q);
  const double m = std::min<double>(S, q.m_max);
  const double passes = S * (m + q.p + q.c + 6.0);
  int rows, nw;
  plan_rows(q.nx, q.ny, g, &rows, &nw);
  const double per_wg = std::max((double)rows * q.nx * ((double)q.n / ((double)q.nx * q.ny)),
                                 md.e_min);
  const double stream = 8.0 * passes * per_wg / md.bw_wg;
  const double serial = S * (md.t_step + (g > 1 ? md.t_team : 0.0) + std::log2((double)g) * md.t_log);
  const double expm = (std::ceil(S / m) + md.rejects) * md.t_expm64 * (m * m) / (64.0 * 64.0);
  return stream + serial + expm;
}

namespace detail {

struct Slot {
  double t;
  int team;
  bool operator>(const Slot& o) const { return t > o.t || (t == o.t && team > o.team); }
};
using MinHeap = std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>>;

// LPT list scheduling on the team mix; returns the makespan and, when
// assign != nullptr, the team of every problem (in `heavy` order).
inline double lpt(const std::vector<PlanProblem>& qs, const std::vector<int>& heavy,
                  const int* gsz, const int* cnt, int ncls, const PlanModel& md,
                  std::vector<int>* assign) {
  MinHeap heaps[3];
  int base = 0;
  for (int c = 0; c < ncls; ++c) {
    for (int i = 0; i < cnt[c]; ++i) heaps[c].push(Slot{0.0, base + i});
    base += cnt[c];
  }
  double makespan = 0.0;
  if (assign) assign->assign(qs.size(), -1);
  for (int idx : heavy) {
    const PlanProblem& q = qs[idx];
    int best_c = -1;
    double best_t = 0.0;
    for (int c = 0; c < ncls; ++c) {
      if (heaps[c].empty()) continue;
      const double f = heaps[c].top().t + plan_time(q, gsz[c], md);
      if (best_c < 0 || f < best_t) {
        best_c = c;
        best_t = f;
      }
    }
    Slot s = heaps[best_c].top();
    heaps[best_c].pop();
    s.t = best_t;
    heaps[best_c].push(s);
    if (assign) (*assign)[idx] = s.team;
    makespan = std::max(makespan, best_t);
  }
  return makespan;
}

}  // namespace detail

// Plan nprob problems on a grid of n_wg workgroups.  Deterministic.
inline Plan make_plan(const std::vector<PlanProblem>& qs, int n_wg, const PlanModel& md) {
  Plan best;
  const int np = (int)qs.size();
  if (np == 0 || n_wg < 1) return best;
  std::vector<int> heavy(np);
  for (int i = 0; i < np; ++i) heavy[i] = i;
  std::vector<double> w1(np);
  for (int i = 0; i < np; ++i) w1[i] = plan_time(qs[i], 1, md);
  std::stable_sort(heavy.begin(), heavy.end(), [&](int a, int b) { return w1[a] > w1[b]; });

  static const int kSizes[] = {2, 4, 8, 16, 32, 64};
  double best_ms = -1.0;
  int bg = 1, bk = 0, mg = 1, mk = 0;
  auto consider = [&](int gb, int kb, int gm, int km) {
    const int ones = n_wg - gb * kb - gm * km;
    if (ones < 0) return;
    int gsz[3], cnt[3], nc = 0;
    if (kb > 0) { gsz[nc] = gb; cnt[nc++] = kb; }
    if (km > 0) { gsz[nc] = gm; cnt[nc++] = km; }
    if (ones > 0) { gsz[nc] = 1; cnt[nc++] = ones; }
    if (nc == 0) return;
    const double ms = detail::lpt(qs, heavy, gsz, cnt, nc, md, nullptr);
    if (best_ms < 0.0 || ms < best_ms * (1.0 - 1e-9)) {
      best_ms = ms;
      bg = gb; bk = kb; mg = gm; mk = km;
    }
  };
  consider(1, 0, 1, 0);
  for (int gb : kSizes) {
    if (gb > n_wg) break;
    const int kb_max = n_wg / gb;
    const int kb_step = std::max(1, kb_max / 32);
    for (int kb = 1; kb <= kb_max; kb += kb_step) {
      consider(gb, kb, 1, 0);
      for (int gm : kSizes) {
        if (gm >= gb) break;
        const int km_max = (n_wg - gb * kb) / gm;
        const int km_step = std::max(1, km_max / 16);
        for (int km = km_step; km <= km_max; km += km_step) consider(gb, kb, gm, km);
      }
    }
  }

  // materialise the winner: teams big, then mid, then single workgroups
  int gsz[3], cnt[3], nc = 0;
  if (bk > 0) { gsz[nc] = bg; cnt[nc++] = bk; }
  if (mk > 0) { gsz[nc] = mg; cnt[nc++] = mk; }
  const int ones = n_wg - bg * bk - mg * mk;
  if (ones > 0) { gsz[nc] = 1; cnt[nc++] = ones; }
  std::vector<int> assign;
  best.makespan = detail::lpt(qs, heavy, gsz, cnt, nc, md, &assign);
  best.g_big = bg; best.k_big = bk; best.g_mid = mg; best.k_mid = mk;
  int wg = 0;
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < cnt[c]; ++i) {
      best.team_size.push_back(gsz[c]);
      best.team_wg0.push_back(wg);
      wg += gsz[c];
    }
  const int nt = (int)best.team_size.size();
  best.team_of_wg.assign(n_wg, -1);
  for (int t = 0; t < nt; ++t)
    for (int i = 0; i < best.team_size[t]; ++i) best.team_of_wg[best.team_wg0[t] + i] = t;
  // problems of each team in `heavy` order; teams without problems stay idle
  std::vector<std::vector<int>> lists(nt);
  for (int idx : heavy) lists[assign[idx]].push_back(idx);
  best.team_first.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) {
    best.team_first[t + 1] = best.team_first[t] + (int)lists[t].size();
    for (int idx : lists[t]) best.order.push_back(idx);
  }
  for (int t = 0; t < nt; ++t)
    if (lists[t].empty())
      for (int i = 0; i < best.team_size[t]; ++i) best.team_of_wg[best.team_wg0[t] + i] = -1;
  double w = 0.0;
  for (int i = 0; i < np; ++i) w += w1[i];
  best.work = w;
  return best;
}

}  // namespace kp
