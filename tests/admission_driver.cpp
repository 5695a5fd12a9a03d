// Reads admission scenarios from stdin and prints the decisions of
// gnp::plan_admission (the solve server's admission policy), so that the
// rules can be checked on a CPU.
//
// Input, per scenario:  budget used max_skips head_skips free_slots
//                       nq  (sys bytes) x nq
//                       ni  (sys bytes stamp) x ni
// Output, per scenario: one line per decision ("REUSE q i", "ALLOC q e...",
//                       "REJECT q"), then "END used head_skips".
#include <iostream>

#include "../paper_2406_00809_amd/csrc/admission.hpp"

int main() {
    size_t budget, used;
    int max_skips, head_skips, free_slots;
    while (std::cin >> budget >> used >> max_skips >> head_skips >> free_slots) {
        gnp::AdmissionState st;
        st.budget = budget;
        st.used = used;
        st.max_skips = max_skips;
        st.head_skips = head_skips;
        size_t nq, ni;
        std::cin >> nq;
        std::vector<gnp::AdmitItem> q(nq);
        for (auto &it : q) std::cin >> it.sys >> it.bytes;
        std::cin >> ni;
        std::vector<gnp::IdleItem> idle(ni);
        for (auto &it : idle) std::cin >> it.sys >> it.bytes >> it.stamp;
        for (const auto &d : gnp::plan_admission(st, free_slots, q, idle)) {
            if (d.kind == gnp::AdmitDecision::REUSE) {
                std::cout << "REUSE " << d.qpos << " " << d.idle_pos << "\n";
            } else if (d.kind == gnp::AdmitDecision::REJECT) {
                std::cout << "REJECT " << d.qpos << "\n";
            } else {
                std::cout << "ALLOC " << d.qpos;
                for (size_t e : d.evict) std::cout << " " << e;
                std::cout << "\n";
            }
        }
        std::cout << "END " << st.used << " " << st.head_skips << "\n";
    }
    return 0;
}
