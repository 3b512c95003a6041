// Persistent grouped launches: one launch serves many work items (scenes or
// scene chunks) of one kernel type and size class.  Each item is the
// argument block of an ordinary launch plus its grid shape; virtual blocks
// are numbered item by item (prefix sums) and handed out through a
// work-queue counter, so workgroups stay resident and balance uneven items.
#pragma once
#include <hip/hip_runtime.h>

namespace nursd {

// Workgroups are handed to the 8 XCDs round-robin by linear id.  This maps a
// linear id to a work item so that each XCD gets one contiguous run of work
// items (neighbouring items then share that XCD's L2).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_contiguous(int lin, int total) {
    const int x = lin % kXcds, k = lin / kXcds;
    const int start = x * (total / kXcds) + min(x, total % kXcds);
    return start + k;
}

template <typename Args>
struct Group {
    const Args* items;     // [n] argument blocks
    const int* prefix;     // [n + 1] first virtual block of each item
    const int* gridx;      // [n] blocks along x of each item
    const int* item_of;    // [total] item of each virtual block
    int n;                 // items
    int total;             // virtual blocks
    int* counter;          // work queue, zeroed before the launch
    int mode;              // kQueue, kStatic or kFlat
};

constexpr int kQueue = 0;   // persistent workgroups dequeue virtual blocks from the counter
constexpr int kStatic = 1;  // persistent workgroups take every gridDim-th virtual block
constexpr int kFlat = 2;    // one workgroup per virtual block (hardware dispatcher)

// Runs body(args, bx, by) for every virtual block of the group.  Every
// workgroup exits once the counter (or its stride) passes the last virtual
// block.
template <typename Args, typename Body>
__device__ __forceinline__ void persistent_loop(const Group<Args>& g, Body body) {
    if (g.mode != kQueue) {
        const int step = g.mode == kFlat ? g.total : (int)gridDim.x;
        for (int vb = blockIdx.x; vb < g.total; vb += step) {
            const int lo = __builtin_amdgcn_readfirstlane(g.item_of[vb]);
            const Args a = g.items[lo];
            const int local = vb - g.prefix[lo];
            const int gx = g.gridx[lo];
            body(a, local % gx, local / gx);
            if (g.mode == kStatic) __syncthreads();
        }
        return;
    }
    __shared__ int s_vb;
    for (;;) {
        if (threadIdx.x == 0) s_vb = atomicAdd(g.counter, 1);
        __syncthreads();
        const int vb = __builtin_amdgcn_readfirstlane(s_vb);
        __syncthreads();
        if (vb >= g.total) break;
        const int lo = __builtin_amdgcn_readfirstlane(g.item_of[vb]);
        const Args a = g.items[lo];
        const int local = vb - g.prefix[lo];
        const int gx = g.gridx[lo];
        body(a, local % gx, local / gx);
        __syncthreads();
    }
}

}  // namespace nursd
