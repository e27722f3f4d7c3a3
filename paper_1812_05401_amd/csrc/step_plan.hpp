// How a call to advance a simulation by n steps is split into launches (host only, no device
// code), kept apart from the runtime so it can be checked on its own.
#pragma once

#include <stdint.h>

namespace vplbm {

// Steps one direct enqueue takes at most: the launches take their step offset within the enqueue
// as an int.  Even, so that a chunk is whole two-step launches.
constexpr int kDirectChunk = 1 << 30;

struct StepChunk {
    bool graph;   // replay the captured graph of graph_k steps; else launch n steps directly
    int n;
};

// The next chunk of a call with `remaining` > 0 steps left: graph replays while at least graph_k
// steps remain (graph_k = 0: no graph), then direct enqueues of at most kDirectChunk steps.  The
// chunks of a call add up to its step count, so the host and device step counters agree.
inline StepChunk next_chunk(int64_t remaining, int graph_k)
{
    if (graph_k > 0 && remaining >= graph_k) return {true, graph_k};
    return {false, remaining > kDirectChunk ? kDirectChunk : (int)remaining};
}

}  // namespace vplbm
