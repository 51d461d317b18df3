// The Arnoldi process of a whole batch in one persistent launch (the
// batching form over problems of uneven size; Sec. 4.3 for the step).
//
// The per-stage launches of the batched solve -- the sketch of R0 (tile),
// beta = ||S(R0)|| (Gram), V_1 (tile), then per step j the sketched inner
// products with the Hessenberg update (Gram), W = Phi(V_j) (operator) and
// V_{j+1} with its two sketches (tile) -- become tasks of one grid of
// resident workgroups.  The problems are cut into eight contiguous groups
// of about equal size (tensor elements), one per XCD (workgroups reach the
// XCDs round-robin, and each XCD has its own L2: neighbouring operator
// tiles share halos, one problem's tiles share its sketch matrices); the
// queue of XCD x holds the tiles of its problems of every stage, stage after
// stage in launch order, and the workgroups of that XCD claim its tasks in
// order from the queue's counter.  Each stage of a
// problem waits only for that problem's own earlier stages:
//
//   sketch of R0   after the operator on X0 (R0 = C - Phi(X0), when given)
//   beta           after the sketch of R0
//   V_1            after beta
//   Gram, step j   after the tiles that formed V_j (its sketch partials)
//   operator, j    after the tiles that formed V_j (W is free again)
//   V_{j+1}        after the Gram step j (coefficients) and the operator j
//
// so the tail of one problem's stage overlaps the next stage of the others
// instead of every stage ending at a grid-wide boundary.  Every task, also
// one that returns early (an inactive problem), adds one to its problem's
// count of finished tasks of its kind; a dependency is a count reaching
// (stages of that kind) x (tiles of the problem per stage).  The Gram
// stage's last workgroup counts itself only after the step's small float64
// part, so a finished Gram count means the step's coefficients are stored.
//
// No deadlock: take the unfinished task that comes first in stage order.
// Its dependencies (earlier stages) are finished.  Every task before it in
// its queue comes earlier in stage order, so is finished too: either a
// workgroup holds it, or the queue's next claim returns it, and every queue
// has workgroups (the grid is a multiple of eight).  A workgroup claims its
// next task while running the current one; the one it holds ahead comes
// after its current task, so the argument stands.
//
// Memory ordering across workgroups (and across the chip's XCDs, whose L2
// caches are separate): every wave waits until its stores are complete, and
// after the workgroup's barrier one release at agent scope (a write-back of
// the XCD's L2) precedes the counts it publishes; a waiting workgroup
// acquires at agent scope after the count is met.  Every wait is bounded: after wait_limit
// polls the workgroup raises the batch's error word, every workgroup stops
// claiming, and the last one to leave marks every problem with
// RTG_F_TIMEOUT, no steps and no further work (the solve that follows
// returns X = X0).
#include "phi_body.h"
#include "tile_body.h"
#include "gram_body.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace rtg {

namespace {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int R, bool TP, bool MB>
struct PersistLds {
    static constexpr int PHI = PhiLayout<R, 4, SL_VEC>::FLOATS * 4;
    static constexpr int TILE = cmax((int)sizeof(TileShared<MB, false, 4>), (int)sizeof(TileShared<MB, MB, 4>));
    static constexpr int BYTES = cmax(cmax(PHI, TILE), (int)sizeof(GramSmem));
};

// A task: stage kind, mode and argument, index within the stage's tiles.
struct Task {
    int kind, mode, arg, b;
    int dep_n[NKIND];   // finished stages of each kind it waits for (0: none)
};

// The tiles of a stage of kind k that queue x takes: those of its problems,
// [qfirst[k][x], qfirst[k][x + 1]).
__device__ __forceinline__ int q_first(const PersistArgs& a, int k, int x) { return a.qfirst[k][x]; }
__device__ __forceinline__ int q_len(const PersistArgs& a, int k, int x) { return a.qfirst[k][x + 1] - a.qfirst[k][x]; }

// Tasks of queue x in their order: [operator on X0], sketch of R0, beta, V_1,
// then per step j = 1..steps the Gram step and, for the first `full` steps,
// the operator and the new basis tensor.
__device__ __forceinline__ int queue_tasks(const PersistArgs& a, int x) {
    const int tp = q_len(a, KIND_PHI, x), tt = q_len(a, KIND_TILE, x), tg = q_len(a, KIND_GRAM, x);
    return (a.any_x0 ? tp : 0) + 2 * tt + tg + a.steps * tg + a.full * (tp + tt);
}

// Task u of queue x (u < queue_tasks(a, x)).
__device__ __forceinline__ Task decode(const PersistArgs& a, int x, int u) {
    Task k;
    k.dep_n[KIND_PHI] = k.dep_n[KIND_TILE] = k.dep_n[KIND_GRAM] = 0;
    const int tp = q_len(a, KIND_PHI, x), tt = q_len(a, KIND_TILE, x), tg = q_len(a, KIND_GRAM, x);
    const int fp = q_first(a, KIND_PHI, x), ft = q_first(a, KIND_TILE, x), fg = q_first(a, KIND_GRAM, x);
    const int x0 = a.any_x0 ? 1 : 0;
    if (x0) {
        if (u < tp) {
            k.kind = KIND_PHI; k.mode = PS_X0; k.arg = 0; k.b = fp + u;
            return k;
        }
        u -= tp;
    }
    if (u < tt) {
        k.kind = KIND_TILE; k.mode = TM_SKETCH_SRC; k.arg = 0; k.b = ft + u;
        k.dep_n[KIND_PHI] = x0;
        return k;
    }
    u -= tt;
    if (u < tg) {
        k.kind = KIND_GRAM; k.mode = GM_START; k.arg = a.cycle; k.b = fg + u;
        k.dep_n[KIND_TILE] = 1;
        return k;
    }
    u -= tg;
    if (u < tt) {
        k.kind = KIND_TILE; k.mode = TM_NEWV; k.arg = 0; k.b = ft + u;
        k.dep_n[KIND_GRAM] = 1;
        return k;
    }
    u -= tt;
    const int per = tg + tp + tt;
    const int j = 1 + u / per;
    u -= (j - 1) * per;
    if (u < tg) {
        k.kind = KIND_GRAM; k.mode = GM_STEP; k.arg = j; k.b = fg + u;
        k.dep_n[KIND_TILE] = j + 1;
        return k;
    }
    u -= tg;
    if (u < tp) {
        k.kind = KIND_PHI; k.mode = PS_BASIS; k.arg = j - 1; k.b = fp + u;
        k.dep_n[KIND_TILE] = j + 1;
        return k;
    }
    u -= tp;
    k.kind = KIND_TILE; k.mode = TM_NEWV; k.arg = j; k.b = ft + u;
    k.dep_n[KIND_GRAM] = j + 1;
    k.dep_n[KIND_PHI] = x0 + j;
    return k;
}

__device__ __forceinline__ int ld_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one thread) until counter >= target; false if the batch's error
// word is raised meanwhile or the wait exceeds the poll limit (which then
// raises it).
__device__ __forceinline__ bool wait_count(const int* counter, int target, int* err, int limit) {
    for (int it = 0;; ++it) {
        if (ld_agent(counter) >= target) return true;
        if (ld_agent(err) != 0) return false;
        if (it >= limit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// two workgroups per CU (the Gram stage's LDS allows no more; the tile
// stage's registers need as many as two waves per SIMD leave)
// Completed tasks whose count is not yet published: each workgroup holds
// up to PEND of them (per counter, how many tasks it gets) and publishes
// them together after one release -- when it holds PEND, before any wait
// that is not already met, and before it leaves.  A workgroup never waits
// while holding unpublished tasks, so the order argument above still holds;
// one L2 write-back then covers several tasks.
constexpr int PEND = 4;

struct Pending {
    int* ctr[PEND];
    int n[PEND];
    int used;   // distinct counters
    int held;   // tasks
};

// one thread: publish every pending count after one release at agent scope
__device__ __forceinline__ void publish(Pending& pd) {
    if (pd.used == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int i = 0; i < pd.used; ++i)
        __hip_atomic_fetch_add(pd.ctr[i], pd.n[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pd.used = 0;
    pd.held = 0;
}

// The descriptors come as a kernel argument of their own, declared
// __restrict__ (the kernel writes through the pointers they hold, never into
// them): their fields are then read by scalar loads, and the buffer resources
// built from them stay in scalar registers.  Read through the argument
// struct, they were vector loads, and every buffer access was wrapped in a
// loop over the lanes' distinct resources.
template <int R, bool TP, bool MB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_persist(PersistArgs a, const Desc* __restrict__ descs) {
    using LY = PersistLds<R, TP, MB>;
    __shared__ __attribute__((aligned(16))) unsigned char lds[LY::BYTES];
    __shared__ int s_task;
    __shared__ Pending s_pend;   // thread 0's list
    const int tid = threadIdx.x;
    int* sched = a.sched;
    // queue of this workgroup: its XCD (workgroups are dispatched to the
    // eight XCDs round-robin), so that a stage's neighbouring tiles -- shared
    // operator halos, one problem's sketch matrices -- meet in one L2
    const int x = blockIdx.x & 7;
    int* next = sched + SCH_QUEUE + SCH_QSTRIDE * x;
    const int ntask = queue_tasks(a, x);
    int claimed = 0;   // thread 0: the task claimed ahead
    if (tid == 0) {
        s_pend.used = 0;
        s_pend.held = 0;
        claimed = __hip_atomic_fetch_add(next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (;;) {
        if (tid == 0) {
            int t = claimed;
            if (t < ntask) claimed = __hip_atomic_fetch_add(next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t >= ntask || ld_agent(sched + SCH_ERROR) != 0) {
                t = -1;
            } else {
                const Task k = decode(a, x, t);
                const int* starts = a.starts[k.kind];
                const int p = find_problem(starts, a.count, k.b);
                const Desc& d = descs[p];
#pragma unroll
                for (int q = 0; q < NKIND; ++q) {
                    const int* ctr = d.state + ST_DONE + q;
                    const int target = k.dep_n[q] * d.ntile[q];
                    if (t < 0 || k.dep_n[q] == 0 || ld_agent(ctr) >= target) continue;
                    publish(s_pend);   // nothing held while waiting
                    if (!wait_count(ctr, target, sched + SCH_ERROR, a.wait_limit)) t = -1;
                }
            }
            s_task = t;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_task);
        if (t < 0) break;
        // the producers' stores (released before they counted in) are seen
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        Task k = decode(a, x, t);
        k.kind = uniform_int(k.kind);
        k.mode = uniform_int(k.mode);
        k.arg = uniform_int(k.arg);
        k.b = uniform_int(k.b);
        const int* starts = uniform_ptr(a.starts[k.kind]);
        if (k.kind == KIND_PHI) {
            phi_batched_task<R, false, 4, false, SL_VEC, TP>(descs, starts, a.count, k.mode, k.arg, k.b,
                                                             (float*)lds);
        } else if (k.kind == KIND_TILE) {
            // a float32 source in the mixed form is split into two bfloat16
            // planes (R0); new basis tensors take one plane
            if (MB && k.mode == TM_SKETCH_SRC)
                tile_task<false, MB, MB, 4>(descs, starts, a.count, k.mode, 0, 0, 0, k.b,
                                            *(TileShared<MB, MB, 4>*)lds);
            else
                tile_task<false, MB, false, 4>(descs, starts, a.count, k.mode, k.arg, k.arg, 0, k.b,
                                               *(TileShared<MB, false, 4>*)lds);
        } else {
            gram_task<false>(descs, starts, a.count, k.mode, k.arg, nullptr, k.b, *(GramSmem*)lds);
        }
        // every wave's stores are complete (in this XCD's L2) before the
        // barrier; then one write-back of the L2 (wave 0's release at agent
        // scope) makes all of them visible to the other XCDs before the task
        // is counted in
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        if (tid == 0) {
            int* ctr = descs[find_problem(starts, a.count, k.b)].state + ST_DONE + k.kind;
            Pending& pd = s_pend;
            int i = 0;
            while (i < pd.used && pd.ctr[i] != ctr) ++i;
            if (i == pd.used) {   // a new counter (held < PEND, so there is room)
                pd.ctr[i] = ctr;
                pd.n[i] = 0;
                pd.used = i + 1;
            }
            pd.n[i] += 1;
            if (++pd.held == PEND) publish(pd);
        }
    }
    // the last workgroup to leave marks every problem of an abandoned batch
    if (tid == 0) {
        publish(s_pend);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int left = __hip_atomic_fetch_add(sched + SCH_EXITED, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == (int)gridDim.x - 1 && ld_agent(sched + SCH_ERROR) != 0) {
            for (int p = 0; p < a.count; ++p) {
                int* st = descs[p].state;
                st[ST_FLAGS] |= RTG_F_TIMEOUT;
                st[ST_MEFF] = 0;
                st[ST_ACTIVE] = 0;
            }
        }
    }
}

struct GridCache {
    std::mutex mu;
    std::map<std::pair<int, const void*>, int> blocks;   // (device, kernel) -> resident workgroups
};

GridCache& grid_cache() {
    static GridCache c;
    return c;
}

template <int R, bool TP, bool MB>
hipError_t launch_one(const PersistArgs& a, hipStream_t s) {
    const void* fn = (const void*)k_persist<R, TP, MB>;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int resident = 0;
    {
        GridCache& gc = grid_cache();
        std::lock_guard<std::mutex> lock(gc.mu);
        auto it = gc.blocks.find({dev, fn});
        if (it != gc.blocks.end()) {
            resident = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            resident = std::max(1, per_cu) * std::max(1, cus);
            gc.blocks[{dev, fn}] = resident;
        }
    }
    // every queue needs a workgroup: a multiple of eight, at least eight
    const int grid = std::max(8, resident & ~7);
    hipLaunchKernelGGL((k_persist<R, TP, MB>), dim3(grid), dim3(256), 0, s, a, a.descs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_persist(const PersistArgs& a, int rmax, int toeplitz, int sketch_bf16, hipStream_t s) {
    const int tier = rmax <= 4 ? 4 : (rmax <= 8 ? 8 : 12);
#define RTG_PERSIST_T(RR)                                            \
    if (toeplitz) {                                                  \
        if (sketch_bf16) return launch_one<RR, true, true>(a, s);    \
        return launch_one<RR, true, false>(a, s);                    \
    }                                                                \
    if (sketch_bf16) return launch_one<RR, false, true>(a, s);       \
    return launch_one<RR, false, false>(a, s);
    if (tier == 4) { RTG_PERSIST_T(4) }
    if (tier == 8) { RTG_PERSIST_T(8) }
    RTG_PERSIST_T(12)
#undef RTG_PERSIST_T
}

}  // namespace rtg
