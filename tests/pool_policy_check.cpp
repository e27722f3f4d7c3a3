// Host check of the serving pool's admission policy (paper_1812_05401_amd/csrc/pool_policy.hpp):
// a first-come-first-served queue driven by may_admit, as the pool drives it between launches.
// Prints one line per scenario: the request ids resident after each event.
#include <cstdio>
#include <deque>
#include <vector>

#include "pool_policy.hpp"

using vplbm::AdmissionState;
using vplbm::may_admit;

struct Req { int id; uint64_t bytes, nodes; };

struct Pool {
    uint64_t budget, max_nodes;
    int slots;
    std::deque<Req> queue;
    std::vector<Req> resident;

    void admit()
    {
        while (!queue.empty()) {
            uint64_t used = 0, nodes = 0;
            for (const Req &r : resident) { used += r.bytes; nodes += r.nodes; }
            const AdmissionState s{used, budget, nodes, max_nodes, slots - (int)resident.size()};
            if (!may_admit(s, queue.front().bytes, queue.front().nodes)) break;
            resident.push_back(queue.front());
            queue.pop_front();
        }
    }
    void retire(int id)
    {
        for (size_t i = 0; i < resident.size(); i++)
            if (resident[i].id == id) { resident.erase(resident.begin() + i); return; }
    }
    void print() const
    {
        std::printf(" [");
        for (size_t i = 0; i < resident.size(); i++) std::printf(i ? ",%d" : "%d", resident[i].id);
        std::printf("]");
    }
};

static Pool make(uint64_t budget, uint64_t max_nodes, int slots, std::vector<Req> reqs)
{
    Pool p{budget, max_nodes, slots, {}, {}};
    for (const Req &r : reqs) p.queue.push_back(r);
    return p;
}

int main()
{
    {   // the budget binds, and the head blocks smaller requests behind it
        Pool p = make(100, 0, 8, {{0, 60, 1}, {1, 50, 1}, {2, 30, 1}});
        std::printf("budget");
        p.admit(); p.print();
        p.retire(0); p.admit(); p.print();
        std::printf("\n");
    }
    {   // the slots bind
        Pool p = make(1000, 0, 2, {{0, 1, 1}, {1, 1, 1}, {2, 1, 1}});
        std::printf("slots");
        p.admit(); p.print();
        p.retire(1); p.admit(); p.print();
        std::printf("\n");
    }
    {   // the node cap binds while something is resident
        Pool p = make(1000, 1000, 8, {{0, 1, 600}, {1, 1, 600}, {2, 1, 100}});
        std::printf("cap");
        p.admit(); p.print();
        p.retire(0); p.admit(); p.print();
        std::printf("\n");
    }
    {   // a request larger than the cap runs alone
        Pool p = make(1000, 1000, 8, {{0, 1, 5000}, {1, 1, 10}});
        std::printf("oversized");
        p.admit(); p.print();
        p.retire(0); p.admit(); p.print();
        std::printf("\n");
    }
    {   // no cap
        Pool p = make(1000, 0, 8, {{0, 1, 600}, {1, 1, 600}, {2, 1, 600}});
        std::printf("nocap");
        p.admit(); p.print();
        std::printf("\n");
    }
    return 0;
}
