// Static list schedule of the tiled factorisation of [Q | I] (host side).
//
// The factorisation of Q = U^T U by 64 x 64 tiles, with the same row
// operations applied to an identity block so that L^-1 = U^-T comes out too,
// is a graph of tile tasks (nt = P / 64 tiles per side):
//   POTRF(k)        factor diagonal tile (k, k): U_kk, D_k = U_kk^-1, L^-1_kk = D_k^T
//   TRSM_U(k, j)    U_kj = D_k^T A_kj                        (j > k)
//   TRSM_L(k, j)    L^-1_kj = D_k^T L^-1_kj                   (j < k)
//   GEMM_U(k, i, j) A_ij -= U_ki^T U_kj                       (k < i <= j)
//   GEMM_L(k, i, j) L^-1_ij -= U_ki^T L^-1_kj                 (j <= k < i)
// Each tile receives its updates in step order and is then finalised by one
// TRSM or POTRF.  The device tracks, per tile, how many of those have been
// applied (a version counter), and every task waits for exactly the versions
// it reads.
//
// The schedule is built once per sampler: a list-scheduling simulation over
// the group's blocks (highest remaining critical path first, earliest-free
// block) with rough task costs.  Every block then runs its list in order.  A
// task starts in the simulation only after its inputs finished, so the lists
// follow one global topological order and the blocks cannot deadlock,
// whatever the real durations are.
#include <algorithm>
#include <cstdint>
#include <queue>
#include <vector>

#include "hsp_internal.hpp"

namespace hsp {

namespace {

struct Task {
    uint32_t code;
    double cost;
    std::vector<uint32_t> succ;
    uint32_t ndep = 0;
    double prio = 0.0;  // longest path from the start of this task to the end
};

}  // namespace

void chol_schedule(uint32_t nt, uint32_t gp, std::vector<uint32_t>* tasks,
                   std::vector<uint32_t>* off) {
    const double c_potrf = 6.0, c_trsm = 1.0, c_gemm = 1.0;
    std::vector<Task> t;
    // ids: potrf[k], trsm_u[k][j], trsm_l[k][j], gemm_u[k][i][j], gemm_l[k][i][j]
    auto idx3 = [nt](uint32_t k, uint32_t i, uint32_t j) { return ((size_t)k * nt + i) * nt + j; };
    std::vector<int64_t> potrf(nt, -1), trsm_u((size_t)nt * nt, -1), trsm_l((size_t)nt * nt, -1);
    std::vector<int64_t> gemm_u((size_t)nt * nt * nt, -1), gemm_l((size_t)nt * nt * nt, -1);
    auto add = [&t](uint32_t code, double cost) {
        t.push_back(Task{code, cost, {}, 0, 0.0});
        return (int64_t)t.size() - 1;
    };
    for (uint32_t k = 0; k < nt; ++k) {
        potrf[k] = add(task_code(kTaskPotrf, 0, k, k, k), c_potrf);
        for (uint32_t j = k + 1; j < nt; ++j) trsm_u[k * nt + j] = add(task_code(kTaskTrsm, 0, k, k, j), c_trsm);
        for (uint32_t j = 0; j < k; ++j) trsm_l[k * nt + j] = add(task_code(kTaskTrsm, 1, k, k, j), c_trsm);
        for (uint32_t i = k + 1; i < nt; ++i) {
            for (uint32_t j = i; j < nt; ++j) gemm_u[idx3(k, i, j)] = add(task_code(kTaskGemm, 0, k, i, j), c_gemm);
            for (uint32_t j = 0; j <= k; ++j) gemm_l[idx3(k, i, j)] = add(task_code(kTaskGemm, 1, k, i, j), c_gemm);
        }
    }
    auto dep = [&t](int64_t from, int64_t to) {
        t[from].succ.push_back((uint32_t)to);
        t[to].ndep++;
    };
    for (uint32_t k = 0; k < nt; ++k) {
        if (k > 0) dep(gemm_u[idx3(k - 1, k, k)], potrf[k]);
        for (uint32_t j = k + 1; j < nt; ++j) {
            dep(potrf[k], trsm_u[k * nt + j]);
            if (k > 0) dep(gemm_u[idx3(k - 1, k, j)], trsm_u[k * nt + j]);
        }
        for (uint32_t j = 0; j < k; ++j) {
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
            for (uint32_t j = 0; j <= k; ++j) {
                const int64_t g = gemm_l[idx3(k, i, j)];
                dep(trsm_u[k * nt + i], g);
                dep(j == k ? potrf[k] : trsm_l[k * nt + j], g);
                if (k > j) dep(gemm_l[idx3(k - 1, i, j)], g);
            }
        }
    }
    // priorities: tasks were created in a topological order, so one reverse pass
    for (size_t n = t.size(); n-- > 0;) {
        double m = 0.0;
        for (uint32_t s : t[n].succ) m = std::max(m, t[s].prio);
        t[n].prio = t[n].cost + m;
    }
    // list scheduling
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
    std::priority_queue<Ready> ready;
    std::priority_queue<Pending> pending;
    std::priority_queue<Worker> workers;
    std::vector<double> ready_at(t.size(), 0.0);
    for (uint32_t n = 0; n < t.size(); ++n)
        if (t[n].ndep == 0) pending.push(Pending{0.0, n});
    for (uint32_t b = 0; b < gp; ++b) workers.push(Worker{0.0, b});
    std::vector<std::vector<uint32_t>> lists(gp);
    size_t done = 0;
    while (done < t.size()) {
        Worker w = workers.top();
        workers.pop();
        double now = w.free;
        if (ready.empty() && !pending.empty() && pending.top().at > now) now = pending.top().at;
        while (!pending.empty() && pending.top().at <= now) {
            ready.push(Ready{t[pending.top().id].prio, pending.top().id});
            pending.pop();
        }
        const uint32_t id = ready.top().id;
        ready.pop();
        const double fin = now + t[id].cost;
        lists[w.b].push_back(t[id].code);
        ++done;
        for (uint32_t s : t[id].succ) {
            ready_at[s] = std::max(ready_at[s], fin);
            if (--t[s].ndep == 0) pending.push(Pending{ready_at[s], s});
        }
        workers.push(Worker{fin, w.b});
    }
    tasks->clear();
    off->assign(1, 0u);
    for (uint32_t b = 0; b < gp; ++b) {
        tasks->insert(tasks->end(), lists[b].begin(), lists[b].end());
        off->push_back((uint32_t)tasks->size());
    }
}

}  // namespace hsp
