// Admission policy of the solve server: which queued requests start now.
//
// Plain host C++ (no HIP), so that the rules can be exercised on a CPU.
//
// A request needs one slot (the server's concurrency limit) and one solve
// workspace for its system (Krylov basis V, network outputs Z, activations,
// residual, right-hand side and solution: the bytes the server reserves in
// HBM).  Finished requests leave their workspace behind, idle and resident,
// so that the next request on the same system starts without allocating.
//
// Rules, applied to the queue in arrival order:
//   1. a request whose workspace alone exceeds the budget can never run: it
//      is rejected;
//   2. an idle workspace of the same system is reused (no new bytes);
//   3. otherwise a new workspace is allocated if it fits in the budget, after
//      evicting idle workspaces of other systems, least recently used first,
//      when that makes it fit;
//   4. a request that does not fit waits (busy workspaces are never
//      evicted).  Later requests that do fit may start ahead of it, but only
//      `max_skips` of them while the same request waits at the head of the
//      queue; after that admission stops until the head fits, so a large
//      request is not starved by a stream of small ones.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace gnp {

struct AdmitItem {
    int sys;       // registered system id
    size_t bytes;  // workspace bytes a new workspace for this system needs
};

struct IdleItem {
    int sys;
    size_t bytes;
    uint64_t stamp;  // larger = used more recently
};

struct AdmitDecision {
    enum Kind { REUSE, ALLOC, REJECT } kind;
    size_t qpos;                // position in the queue given to plan()
    size_t idle_pos;            // REUSE: position in the idle list given to plan()
    std::vector<size_t> evict;  // ALLOC: idle positions to free first
};

struct AdmissionState {
    size_t budget = 0;  // HBM bytes the server may hold in workspaces
    size_t used = 0;    // bytes held by busy and idle workspaces
    int head_skips = 0; // admissions made past the current blocked head
    int max_skips = 8;
};

// Decide which queued requests start now.  `free_slots` is the number of
// idle slots.  Positions in the result refer to `queue` and `idle` as given;
// st.used and st.head_skips are updated as if the decisions were applied.
inline std::vector<AdmitDecision> plan_admission(AdmissionState &st, int free_slots,
                                                 const std::vector<AdmitItem> &queue,
                                                 const std::vector<IdleItem> &idle) {
    std::vector<AdmitDecision> out;
    std::vector<bool> taken(idle.size(), false);  // reused or evicted
    bool head_blocked = false;
    for (size_t q = 0; q < queue.size(); ++q) {
        const AdmitItem &it = queue[q];
        if (it.bytes > st.budget) {  // rule 1 (needs no slot)
            out.push_back({AdmitDecision::REJECT, q, 0, {}});
            continue;
        }
        if (free_slots <= 0) break;
        if (head_blocked && st.head_skips >= st.max_skips) break;
        // rule 2: most recently used idle workspace of the same system
        size_t best = idle.size();
        for (size_t k = 0; k < idle.size(); ++k)
            if (!taken[k] && idle[k].sys == it.sys &&
                (best == idle.size() || idle[k].stamp > idle[best].stamp))
                best = k;
        if (best < idle.size()) {
            taken[best] = true;
            out.push_back({AdmitDecision::REUSE, q, best, {}});
            --free_slots;
            if (head_blocked) ++st.head_skips;
            continue;
        }
        // rule 3: allocate, evicting least recently used idle workspaces of
        // other systems if that makes the request fit
        std::vector<size_t> evict;
        if (st.used + it.bytes > st.budget) {
            std::vector<size_t> order;
            for (size_t k = 0; k < idle.size(); ++k)
                if (!taken[k]) order.push_back(k);
            std::sort(order.begin(), order.end(),
                      [&](size_t a, size_t b) { return idle[a].stamp < idle[b].stamp; });
            size_t freed = 0;
            for (size_t k : order) {
                if (st.used - freed + it.bytes <= st.budget) break;
                evict.push_back(k);
                freed += idle[k].bytes;
            }
            if (st.used - freed + it.bytes > st.budget) {  // rule 4: wait
                if (!head_blocked) {
                    head_blocked = true;
                    if (q != 0) st.head_skips = 0;  // a new request heads the wait
                }
                continue;
            }
            for (size_t k : evict) taken[k] = true;
            st.used -= freed;
        }
        st.used += it.bytes;
        out.push_back({AdmitDecision::ALLOC, q, 0, evict});
        --free_slots;
        if (head_blocked) ++st.head_skips;
    }
    if (!head_blocked) st.head_skips = 0;
    return out;
}

}  // namespace gnp
