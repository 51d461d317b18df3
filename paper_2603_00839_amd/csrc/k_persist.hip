// The Arnoldi process of a whole batch in one persistent launch (the
// batching form over problems of uneven size; Sec. 4.3 for the step).
//
// The per-stage launches of the batched solve -- the sketch of R0 (tile),
// beta = ||S(R0)|| (Gram), V_1 (tile), then per step j the sketched inner
// products with the Hessenberg update (Gram), W = Phi(V_j) (operator) and
// V_{j+1} with its two sketches (tile) -- become tasks of one grid of
// resident workgroups.  Tasks are numbered stage after stage exactly as the
// launches would run them (every problem's tiles of a stage, problem after
// problem), and a workgroup claims the next number from a global counter.
// Each stage of a problem waits only for that problem's own earlier stages:
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
// No deadlock: numbers are claimed in increasing order and every dependency
// has a smaller number, so the smallest unfinished claimed task always has
// its dependencies finished and belongs to a running workgroup.  Each
// workgroup claims its next task while running the current one.
//
// Memory ordering across workgroups (and across the chip's XCDs, whose L2
// caches are separate): every wave releases its stores at agent scope before
// the workgroup counts the task in; a waiting workgroup acquires at agent
// scope after the count is met.  Every wait is bounded: after wait_limit
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

// Task t of the batch (t < total).  Stages: [operator on X0], sketch of R0,
// beta, V_1, then per step j = 1..mmax the Gram step and, unless it is the
// last step without V_{m+1}, the operator and the new basis tensor.
__device__ __forceinline__ Task decode(const PersistArgs& a, int t) {
    Task k;
    k.dep_n[KIND_PHI] = k.dep_n[KIND_TILE] = k.dep_n[KIND_GRAM] = 0;
    const int x0 = a.any_x0 ? 1 : 0;
    if (x0) {
        if (t < a.tp) {
            k.kind = KIND_PHI; k.mode = PS_X0; k.arg = 0; k.b = t;
            return k;
        }
        t -= a.tp;
    }
    if (t < a.tt) {
        k.kind = KIND_TILE; k.mode = TM_SKETCH_SRC; k.arg = 0; k.b = t;
        k.dep_n[KIND_PHI] = x0;
        return k;
    }
    t -= a.tt;
    if (t < a.tg) {
        k.kind = KIND_GRAM; k.mode = GM_START; k.arg = a.cycle; k.b = t;
        k.dep_n[KIND_TILE] = 1;
        return k;
    }
    t -= a.tg;
    if (t < a.tt) {
        k.kind = KIND_TILE; k.mode = TM_NEWV; k.arg = 0; k.b = t;
        k.dep_n[KIND_GRAM] = 1;
        return k;
    }
    t -= a.tt;
    const int per = a.tg + a.tp + a.tt;
    const int j = 1 + t / per;
    t -= (j - 1) * per;
    if (t < a.tg) {
        k.kind = KIND_GRAM; k.mode = GM_STEP; k.arg = j; k.b = t;
        k.dep_n[KIND_TILE] = j + 1;
        return k;
    }
    t -= a.tg;
    if (t < a.tp) {
        k.kind = KIND_PHI; k.mode = PS_BASIS; k.arg = j - 1; k.b = t;
        k.dep_n[KIND_TILE] = j + 1;
        return k;
    }
    t -= a.tp;
    k.kind = KIND_TILE; k.mode = TM_NEWV; k.arg = j; k.b = t;
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
template <int R, bool TP, bool MB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_persist(PersistArgs a) {
    using LY = PersistLds<R, TP, MB>;
    __shared__ __attribute__((aligned(16))) unsigned char lds[LY::BYTES];
    __shared__ int s_task;
    const int tid = threadIdx.x;
    int* sched = a.sched;
    int claimed = 0;   // thread 0: the task claimed ahead
    if (tid == 0) claimed = __hip_atomic_fetch_add(sched + SCH_NEXT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0) {
            int t = claimed;
            if (t < a.total) claimed = __hip_atomic_fetch_add(sched + SCH_NEXT, 1, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
            if (t >= a.total || ld_agent(sched + SCH_ERROR) != 0) {
                t = -1;
            } else {
                const Task k = decode(a, t);
                const int* starts = a.starts[k.kind];
                const int p = find_problem(starts, a.count, k.b);
                const Desc& d = a.descs[p];
#pragma unroll
                for (int q = 0; q < NKIND; ++q)
                    if (t >= 0 && k.dep_n[q] > 0 &&
                        !wait_count(d.state + ST_DONE + q, k.dep_n[q] * d.ntile[q], sched + SCH_ERROR, a.wait_limit))
                        t = -1;
            }
            s_task = t;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_task);
        if (t < 0) break;
        // the producers' stores (released before they counted in) are seen
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const Task k = decode(a, t);
        const int* starts = a.starts[k.kind];
        if (k.kind == KIND_PHI) {
            phi_batched_task<R, false, 4, false, SL_VEC, TP>(a.descs, starts, a.count, k.mode, k.arg, k.b,
                                                             (float*)lds);
        } else if (k.kind == KIND_TILE) {
            // a float32 source in the mixed form is split into two bfloat16
            // planes (R0); new basis tensors take one plane
            if (MB && k.mode == TM_SKETCH_SRC)
                tile_task<false, MB, MB, 4>(a.descs, starts, a.count, k.mode, 0, 0, 0, k.b,
                                            *(TileShared<MB, MB, 4>*)lds);
            else
                tile_task<false, MB, false, 4>(a.descs, starts, a.count, k.mode, k.arg, k.arg, 0, k.b,
                                               *(TileShared<MB, false, 4>*)lds);
        } else {
            gram_task<false>(a.descs, starts, a.count, k.mode, k.arg, nullptr, k.b, *(GramSmem*)lds);
        }
        // every wave's stores reach memory before the task is counted in
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const int p = find_problem(starts, a.count, k.b);
            __hip_atomic_fetch_add(a.descs[p].state + ST_DONE + k.kind, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the last workgroup to leave marks every problem of an abandoned batch
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int left = __hip_atomic_fetch_add(sched + SCH_EXITED, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == (int)gridDim.x - 1 && ld_agent(sched + SCH_ERROR) != 0) {
            for (int p = 0; p < a.count; ++p) {
                int* st = a.descs[p].state;
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
    const int grid = std::max(1, std::min(resident, a.total));
    hipLaunchKernelGGL((k_persist<R, TP, MB>), dim3(grid), dim3(256), 0, s, a);
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
