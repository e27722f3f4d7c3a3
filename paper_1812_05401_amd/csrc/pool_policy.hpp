// Admission policy of the serving pool (host only, no device code): which queued request may
// become resident.  Kept apart from the device bookkeeping so it can be checked on its own.
#pragma once

#include <stdint.h>

namespace vplbm {

struct AdmissionState {
    uint64_t used_bytes;       // device memory charged to the resident simulations
    uint64_t budget_bytes;     // the pool's budget
    uint64_t resident_nodes;   // lattice nodes of the resident simulations
    uint64_t max_nodes;        // admission cap on resident nodes (0: none)
    int free_slots;
};

// Whether a request of `bytes` and `nodes` fits now.  The memory budget and the slots always
// bind; the node cap binds only while something is resident, so a request larger than the cap
// still runs, alone.  Requests are taken first come, first served: a head that does not fit
// blocks the queue until retirements make room.
inline bool may_admit(const AdmissionState &s, uint64_t bytes, uint64_t nodes)
{
    if (s.free_slots <= 0) return false;
    if (s.used_bytes + bytes > s.budget_bytes) return false;
    if (s.max_nodes && s.resident_nodes > 0 && s.resident_nodes + nodes > s.max_nodes) return false;
    return true;
}

// What the pool does when the device refuses a request's memory although the budget admits it: wait
// for retirements while simulations are resident; with none resident nothing will ever be freed,
// so the request fails (VPLBM_FAILED, status 2) instead of blocking the queue for good.
inline bool fail_when_refused(bool anything_resident) { return !anything_resident; }

}  // namespace vplbm
