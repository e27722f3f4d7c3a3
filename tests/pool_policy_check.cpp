// Host check of the serving pool's admission policy (paper_1812_05401_amd/csrc/pool_policy.hpp):
// a first-come-first-served queue driven by may_admit, as the pool drives it between launches.
// Prints one line per scenario: the request ids resident after each event.
#include <cstdio>
#include <deque>
#include <vector>

#include "pool_policy.hpp"
#include "step_plan.hpp"

using vplbm::AdmissionState;
using vplbm::may_admit;

struct Req { int id; uint64_t bytes, nodes; bool refused = false; };

struct Pool {
    uint64_t budget, max_nodes;
    int slots;
    std::deque<Req> queue;
    std::vector<Req> resident;
    std::vector<int> failed;

    // as the pool's advance does: a request the device refuses (refused = true) waits while
    // something is resident and fails when nothing is
    void admit()
    {
        while (!queue.empty()) {
            uint64_t used = 0, nodes = 0;
            for (const Req &r : resident) { used += r.bytes; nodes += r.nodes; }
            const AdmissionState s{used, budget, nodes, max_nodes, slots - (int)resident.size()};
            if (!may_admit(s, queue.front().bytes, queue.front().nodes)) break;
            if (queue.front().refused) {
                if (!vplbm::fail_when_refused(!resident.empty())) break;
                failed.push_back(queue.front().id);
                queue.pop_front();
                continue;
            }
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
        if (!failed.empty()) {
            std::printf("failed:");
            for (size_t i = 0; i < failed.size(); i++) std::printf(i ? ",%d" : "%d", failed[i]);
        }
    }
};

// The chunks vplbm_step would take for n steps with a graph of k steps: prints the number of
// graph replays, the direct chunks, and whether they add up to n with every direct chunk in
// (0, kDirectChunk] and all but the last even.
static void plan(const char *name, int64_t n, int k)
{
    int64_t left = n, replays = 0, sum = 0;
    std::vector<int> direct;
    bool ok = true;
    while (left > 0) {
        const vplbm::StepChunk c = vplbm::next_chunk(left, k);
        if (c.graph) replays++;
        else direct.push_back(c.n);
        ok &= c.n > 0 && c.n <= vplbm::kDirectChunk;
        sum += c.n;
        left -= c.n;
    }
    for (size_t i = 0; i + 1 < direct.size(); i++) ok &= direct[i] % 2 == 0;
    std::printf("%s %lld", name, (long long)replays);
    for (int d : direct) std::printf(" %d", d);
    std::printf(" %s\n", ok && sum == n ? "ok" : "BAD");
}

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
    {   // the device refuses request 1: it waits behind resident 0, then fails once 0 retires
        Pool p = make(1000, 0, 8, {{0, 1, 1}, {1, 1, 1, true}, {2, 1, 1}});
        std::printf("refused");
        p.admit(); p.print();
        p.retire(0); p.admit(); p.print();
        std::printf("\n");
    }
    plan("plan_short", 3, 128);
    plan("plan_graph", 300, 128);
    plan("plan_nograph", 1001, 0);
    plan("plan_2e31", (1LL << 31) + 5, 0);
    plan("plan_2e32_graph", (1LL << 32) + 7, 128);
    return 0;
}
