// Static list schedule of the tiled factorisation of [Q | I] (host side).
// (Beyond p = kSubstP the L^-1 tasks are left out: see with_inverse.)
//
// The factorisation of Q = U^T U by 64 x 64 tiles, with the same row
// operations applied to an identity block so that L^-1 = U^-T comes out too,
// is a graph of tile tasks (nt = P / 64 tiles per side):
//   POTRF(k)        factor diagonal tile (k, k): U_kk, D_k = U_kk^-1, L^-1_kk = D_k^T
//   TRSM_U(k, j)    U_kj = D_k^T A_kj                        (j > k)
//   TRSM_L(k, j)    L^-1_kj = D_k^T L^-1_kj                   (j < k)
//   GEMM_U(k, i, j) A_ij -= U_ki^T U_kj                       (k < i <= j)
//   GEMM_L(k, i, j) L^-1_ij -= U_ki^T L^-1_kj                 (j <= k < i)
//   PANEL(k)        TRSM_U(k-1, k), GEMM_U(k-1, k, k) and POTRF(k) in one block,
//                   D_k-1 and the tiles staying in that block's LDS (k >= 1)
// Each tile receives its updates in step order and is then finalised by one
// TRSM or POTRF.  The chain POTRF(0), PANEL(1), PANEL(2), ... is the
// critical path; block 0 runs it and nothing else.  The device tracks, per tile, how many of those have been
// applied (a version counter), and every task waits for exactly the versions
// it reads.
//
// The schedule is built once per sampler: a list-scheduling simulation over
// the group's other blocks (highest remaining critical path first,
// earliest-free block) with rough task costs orders the tasks.  Block 0 runs
// the chain; the other blocks take the remaining tasks from one shared queue
// in that order, each claiming the next when it is free, so the real task
// durations decide who runs what.  A task starts in the simulation only after
// its inputs finished, so the order is topological: the earliest unfinished
// task always has its inputs and has been claimed by a block that is free to
// run it, and the group cannot deadlock.
#include <algorithm>
#include <cstdint>
#include <queue>
#include <vector>

#include "hsp_internal.hpp"

namespace hsp {

namespace {

constexpr uint32_t kNoTask = 0xffffffffu;  // a simulated-only part of a merged task

struct Task {
    uint32_t code;
    double cost;
    std::vector<uint32_t> succ;
    uint32_t ndep = 0;
    double prio = 0.0;  // longest path from the start of this task to the end
};

}  // namespace

void chol_schedule(uint32_t nt, uint32_t gp, std::vector<uint32_t>* tasks,
                   std::vector<uint32_t>* off, bool inverse) {
    // rough costs in units of one tile task
    const double c_potrf = 3.5, c_panel = 4.5, c_trsm = 1.0, c_gemm = 1.0;
    const bool chain = gp > 1;  // block 0 owns the critical chain
    const bool inv = inverse;  // the L^-1 tasks (TRSM_L, GEMM_L) are part of the graph
    std::vector<Task> t;
    auto idx3 = [nt](uint32_t k, uint32_t i, uint32_t j) { return ((size_t)k * nt + i) * nt + j; };
    // ids: potrf[k] (k = 0, or every k without a chain block), panel[k] (k >= 1 with one),
    // trsm_u[k][j], trsm_l[k][j], gemm_u[k][i][j], gemm_l[k][i][j]; a merged task
    // stands in for the parts it absorbed
    std::vector<int64_t> potrf(nt, -1), trsm_u((size_t)nt * nt, -1), trsm_l((size_t)nt * nt, -1);
    std::vector<int64_t> gemm_u((size_t)nt * nt * nt, -1), gemm_l((size_t)nt * nt * nt, -1);
    std::vector<bool> on_chain;
    std::vector<std::pair<int64_t, int64_t>> panel_first;  // (first half, second half)
    auto add = [&t, &on_chain](uint32_t code, double cost, bool ch) {
        t.push_back(Task{code, cost, {}, 0, 0.0});
        on_chain.push_back(ch);
        return (int64_t)t.size() - 1;
    };
    for (uint32_t k = 0; k < nt; ++k) {
        if (chain && k > 0) {
            // simulated as its two halves: the solve of tile (k-1, k), published
            // as soon as it is done, then the update and factorisation of (k, k)
            const int64_t pa = add(task_code(kTaskPanel, 0, k, k, k), c_trsm, true);
            const int64_t pb = add(kNoTask, c_panel - c_trsm, true);
            potrf[k] = pb;
            trsm_u[(k - 1) * nt + k] = pa;
            gemm_u[idx3(k - 1, k, k)] = pb;
            panel_first.push_back({pa, pb});
        } else {
            potrf[k] = add(task_code(kTaskPotrf, 0, k, k, k), c_potrf, chain);
        }
        for (uint32_t j = k + 1; j < nt; ++j)
            if (!(chain && j == k + 1)) trsm_u[k * nt + j] = add(task_code(kTaskTrsm, 0, k, k, j), c_trsm, false);
        for (uint32_t j = 0; inv && j < k; ++j) trsm_l[k * nt + j] = add(task_code(kTaskTrsm, 1, k, k, j), c_trsm, false);
        for (uint32_t i = k + 1; i < nt; ++i) {
            for (uint32_t j = i; j < nt; ++j)
                if (!(chain && i == k + 1 && j == k + 1))
                    gemm_u[idx3(k, i, j)] = add(task_code(kTaskGemm, 0, k, i, j), c_gemm, false);
            for (uint32_t j = 0; inv && j <= k; ++j)
                gemm_l[idx3(k, i, j)] = add(task_code(kTaskGemm, 1, k, i, j), c_gemm, false);
        }
    }
    // trsm_u[k][k+1] and gemm_u[k][k+1][k+1] are created with step k + 1's panel
    // above only when k + 1 < nt is reached; fill them in before the edges
    std::vector<std::pair<int64_t, int64_t>> edges;
    auto dep = [&edges](int64_t from, int64_t to) {
        if (from != to) edges.emplace_back(from, to);
    };
    for (auto& h : panel_first) dep(h.first, h.second);
    for (uint32_t k = 0; k < nt; ++k) {
        if (k > 0) dep(gemm_u[idx3(k - 1, k, k)], potrf[k]);
        if (chain && k > 0) {
            // the panel reads tiles (k-1, k) and (k, k) at version k-1 and runs
            // after the previous one (both inputs are waited for before its start)
            const int64_t pa = trsm_u[(k - 1) * nt + k];
            if (k > 1) dep(gemm_u[idx3(k - 2, k - 1, k)], pa);
            if (k > 1) dep(gemm_u[idx3(k - 2, k, k)], pa);
            dep(potrf[k - 1], pa);
        }
        for (uint32_t j = k + 1; j < nt; ++j) {
            dep(potrf[k], trsm_u[k * nt + j]);
            if (k > 0) dep(gemm_u[idx3(k - 1, k, j)], trsm_u[k * nt + j]);
        }
        for (uint32_t j = 0; inv && j < k; ++j) {
            dep(potrf[k], trsm_l[k * nt + j]);
            dep(gemm_l[idx3(k - 1, k, j)], trsm_l[k * nt + j]);
        }
        for (uint32_t i = k + 1; i < nt; ++i) {
            for (uint32_t j = i; j < nt; ++j) {
                const int64_t g = gemm_u[idx3(k, i, j)];
                dep(trsm_u[k * nt + i], g);
                if (j != i) dep(trsm_u[k * nt + j], g);
                if (k > 0) dep(gemm_u[idx3(k - 1, i, j)], g);
            }
            for (uint32_t j = 0; inv && j <= k; ++j) {
                const int64_t g = gemm_l[idx3(k, i, j)];
                dep(trsm_u[k * nt + i], g);
                dep(j == k ? potrf[k] : trsm_l[k * nt + j], g);
                if (k > j) dep(gemm_l[idx3(k - 1, i, j)], g);
            }
        }
    }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    for (auto& e : edges) {
        t[e.first].succ.push_back((uint32_t)e.second);
        t[e.second].ndep++;
    }
    // priorities: longest path to the end (tasks are not created in topological
    // order any more, so iterate to a fixed point over the edge list)
    for (auto& x : t) x.prio = x.cost;
    for (bool changed = true; changed;) {
        changed = false;
        for (auto it = edges.rbegin(); it != edges.rend(); ++it) {
            const double v = t[it->first].cost + t[it->second].prio;
            if (v > t[it->first].prio) {
                t[it->first].prio = v;
                changed = true;
            }
        }
    }
    // list scheduling: chain tasks on block 0, the rest on blocks 1.. (or all on
    // block 0 when the group has one block)
    struct Ready {
        double prio;
        uint32_t id;
        bool operator<(const Ready& o) const { return prio < o.prio || (prio == o.prio && id > o.id); }
    };
    struct Pending {
        double at;
        uint32_t id;
        bool operator<(const Pending& o) const { return at > o.at || (at == o.at && id > o.id); }
    };
    struct Worker {
        double free;
        uint32_t b;
        bool operator<(const Worker& o) const { return free > o.free || (free == o.free && b > o.b); }
    };
    std::priority_queue<Ready> ready[2];
    std::priority_queue<Pending> pending[2];
    std::priority_queue<Worker> workers[2];
    std::vector<double> ready_at(t.size(), 0.0);
    auto cls = [&](uint32_t n) { return chain && on_chain[n] ? 0 : 1; };
    for (uint32_t n = 0; n < t.size(); ++n)
        if (t[n].ndep == 0) pending[cls(n)].push(Pending{0.0, n});
    if (chain) {
        workers[0].push(Worker{0.0, 0});
        for (uint32_t b = 1; b < gp; ++b) workers[1].push(Worker{0.0, b});
    } else {
        workers[1].push(Worker{0.0, 0});
    }
    std::vector<std::vector<uint32_t>> lists(gp);
    std::vector<std::pair<double, uint32_t>> order;  // (simulated start, task)
    // Event simulation on one clock that never goes back: at each instant,
    // every free block of a class takes the highest-priority task that is
    // ready by then.  Start times are therefore a topological order.
    size_t done = 0;
    double clock = 0.0;
    const double inf = 1e300;
    while (done < t.size()) {
        for (int c = 0; c < 2; ++c) {
            while (!pending[c].empty() && pending[c].top().at <= clock) {
                ready[c].push(Ready{t[pending[c].top().id].prio, pending[c].top().id});
                pending[c].pop();
            }
            while (!ready[c].empty() && !workers[c].empty() && workers[c].top().free <= clock) {
                const Worker w = workers[c].top();
                workers[c].pop();
                const uint32_t id = ready[c].top().id;
                ready[c].pop();
                const double fin = clock + t[id].cost;
                if (t[id].code != kNoTask) {
                    lists[w.b].push_back(t[id].code);
                    order.push_back({clock, id});
                }
                ++done;
                for (uint32_t s2 : t[id].succ) {
                    ready_at[s2] = std::max(ready_at[s2], fin);
                    if (--t[s2].ndep == 0) pending[cls(s2)].push(Pending{ready_at[s2], s2});
                }
                workers[c].push(Worker{fin, w.b});
            }
        }
        // next instant at which some block can take some task
        double next = inf;
        for (int c = 0; c < 2; ++c) {
            if (workers[c].empty()) continue;
            const double wf = workers[c].top().free;
            if (!ready[c].empty()) next = std::min(next, std::max(wf, clock));
            if (!pending[c].empty()) next = std::min(next, std::max(wf, pending[c].top().at));
        }
        if (next >= inf) break;  // nothing left that can run (cannot happen for a DAG)
        clock = std::max(clock, next);
    }

    // Output: with one block, its list; otherwise block 0's chain list, then
    // every other task in order of simulated start (a topological order,
    // highest priority first among tasks ready together): the queue the other
    // blocks take tasks from, one at a time, as they become free.
    tasks->clear();
    off->assign(1, 0u);
    if (!chain) {
        tasks->insert(tasks->end(), lists[0].begin(), lists[0].end());
        off->push_back((uint32_t)tasks->size());
        return;
    }
    tasks->insert(tasks->end(), lists[0].begin(), lists[0].end());
    off->push_back((uint32_t)tasks->size());
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, uint32_t>& x, const std::pair<double, uint32_t>& y) {
                         return x.first < y.first;
                     });
    for (auto& o : order)
        if (!on_chain[o.second]) tasks->push_back(t[o.second].code);
    off->push_back((uint32_t)tasks->size());
}

}  // namespace hsp
