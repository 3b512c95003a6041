// Persistent grouped launches: one launch serves many work items (scenes or
// scene chunks) of one kernel type and size class.  Each item is the
// argument block of an ordinary launch plus its grid shape; virtual blocks
// are numbered item by item (prefix sums) and handed out through a
// work-queue counter, so workgroups stay resident and balance uneven items.
#pragma once
#include <hip/hip_runtime.h>

namespace nursd {

template <typename Args>
struct Group {
    const Args* items;     // [n] argument blocks
    const int* prefix;     // [n + 1] first virtual block of each item
    const int* gridx;      // [n] blocks along x of each item
    int n;                 // items
    int total;             // virtual blocks
    int* counter;          // work queue, zeroed before the launch
};

// Runs body(args, bx, by) for every virtual block of the group.  Every
// workgroup exits once the counter passes the last virtual block.
template <typename Args, typename Body>
__device__ __forceinline__ void persistent_loop(const Group<Args>& g, Body body) {
    __shared__ int s_vb;
    for (;;) {
        if (threadIdx.x == 0) s_vb = atomicAdd(g.counter, 1);
        __syncthreads();
        const int vb = s_vb;
        __syncthreads();
        if (vb >= g.total) break;
        int lo = 0, hi = g.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.prefix[mid] <= vb) lo = mid; else hi = mid - 1;
        }
        const Args a = g.items[lo];
        const int local = vb - g.prefix[lo];
        const int gx = g.gridx[lo];
        body(a, local % gx, local / gx);
        __syncthreads();
    }
}

}  // namespace nursd
