// Internal declarations shared by the HIP translation units of librtg.so.
//
// One "problem" is one RTG-GMRES solve; a launch covers the tiles of every
// problem of a batch.  Each problem is described by a Desc living in device
// memory; kernels map blockIdx.x to (problem, tile) through per-kernel-kind
// prefix offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/rtg.h"

namespace rtg {

typedef unsigned short bf16_t;   // raw bfloat16 bit pattern

constexpr int RMAX_SPATIAL = 12;   // max half-bandwidth of A1, A2
constexpr int RMAX_B = 8;          // max half-bandwidth of B
constexpr int LMAX_SPATIAL = 128;  // max l1, l2
constexpr int LMAX_3 = 16;         // max l3 when Om3 is given
constexpr int MMAX = 96;           // max Arnoldi steps (FP64 SVD fits in LDS)

// operator tile (k_phi): T1 rows (i1) x T2 columns (i2) x JT (4 or 8) channels
constexpr int PHI_T1 = 64;
constexpr int PHI_T2 = 32;
// AXPY/sketch tile (k_tile): I1 rows x TC columns of one channel
constexpr int TILE_TC = 32;
// sketched-Gram chunk (k_gram): CH (a,b) pairs per workgroup
constexpr int GRAM_CH = 256;

enum KernelKind { KIND_PHI = 0, KIND_TILE = 1, KIND_GRAM = 2, NKIND = 3 };

// state[] slots (int)
// (ST_ITERS: steps of the finished restart cycles; ST_SKIP: this problem sits
// out the current restart cycle, X and its info stay as they are)
// (ST_DONE + kind: tasks of that kind finished for this problem in the
// persistent launch, one slot per KernelKind)
enum { ST_ACTIVE = 0, ST_MEFF = 1, ST_FLAGS = 2, ST_COUNTER = 3, ST_ITERS = 4, ST_SKIP = 5, ST_DONE = 6, NSTATE = 16 };
static_assert(ST_DONE + NKIND <= NSTATE, "state slots");
// scal[] slots (double)
enum { SC_BETA = 0, SC_MU = 1, SC_RESPROJ = 2, SC_RESLS = 3, SC_RHO = 4, NSCAL = 16 };

struct Desc {
    // sizes
    int I1, I2, J;
    int l1, l2, l3;
    int r1, r2, rB;
    int m;              // max steps for this problem
    int bf16;           // basis stored as bfloat16
    int skbf;           // sketch contractions on bfloat16 MFMA operands (a bfloat16 basis, or the
                        // float32 basis of the mixed form RTG_F32_BF16)
    int has_om3;        // Om3 given (else identity, l3 == J)
    int n_i2t;          // ceil(I2 / TILE_TC)
    int ntile[NKIND];   // tiles of this problem per kernel kind
    int mu_fixed;       // 1: mu given, 0: chosen by mu_rule
    int mu_rule;        // RTG_MU_DISCREPANCY or RTG_MU_GCV
    int keep_last;      // form V_{m+1} after the last step (Arnoldi-only calls)
    int toeplitz;       // A1 and A2 are Toeplitz on their in-range entries (convolutions, zero BC)
    int gram_ch;        // (a, b) pairs per sketched-Gram workgroup chosen for the batch (0: the default)
    int unsketched;     // identity sketch: Frobenius inner products of the full tensors
    int restarts;       // restart cycles after the first (restarted RTG-GMRES), 0 = none
    int gk;             // sketched Block Golub-Kahan: 1 = the V side (operator Phi), 2 = the U side
                        // (operator Phi^T, transposed bands); 0 = RTG-GMRES
    int fallback;       // a re-solve by the plain solver after a failed warm-started solve:
                        // RTG_F_FALLBACK is set in its flags from the start
    int lazy_v1;        // V_1 is stored as R0 itself (bfloat16), not R0 / beta: the pass that
                        // forms it also sketches it, and beta = ||S(V_1)|| is applied where
                        // V_1 is used (its sketches, its multi-AXPY coefficient and the
                        // assembly); bfloat16-basis solves with the fused step only
    long long n;        // I1*I2*J
    long long L;        // l1*l2*l3
    // operator / sketch (device)
    const float* a1;
    const float* a2;
    const float* bb;
    const float* a1t;             // bands transposed: a1t[(r1 + dd) I1 + i] = a1[i (2 r1 + 1) + r1 + dd]
    const float* a2t;
    const float* a1p[3];          // A1 band rows zero-padded to the tiers R = 4, 8, 12 (row stride 2R+1 rounded up to 4)
    const float* taps;            // toeplitz: A1 taps at [r1 + dd], A2 taps at [2 RMAX_SPATIAL + 1 + r2 + dd]
    const float* st;              // general PSF: stencil [a + r1][b + r1] (weight of X[i1 + a, i2 + b]),
                                  // r1 = r2; the bands are then absent and the sketch of W = Phi(V) is
                                  // taken from W itself (no composed matrices)
    const float* om1;
    const bf16_t* om1h;           // bfloat16 copy of Om1
    const float* om1f;            // Om1 in operand order, FRAG_K_F32
    const bf16_t* om1hf;          // bfloat16 Om1 in operand order, FRAG_K_BF16
    const float* om2;
    const float* om3;             // nullptr => identity
    // sketch of Phi(X) as a sketch of X (mode products compose, eq. (2)):
    // Om1 A1 (float32, and bfloat16 high then low planes, both in operand
    // order), Om2 A2, Om3 B^T (l3 x J)
    const float* om1t;
    const bf16_t* om1th;
    const float* om2t;
    const float* om3t;
    // data (device)
    const float* C;
    const float* X0;    // nullptr => 0
    float* X;
    const void* R0src;  // tensor whose sketch starts the process (C, W or R0)
    int src_bf16;       // R0src holds bfloat16 (stand-alone sketch only)
    rtg_info* info;
    // workspace (device)
    void* V;            // (m+1) tensors
    float* W;           // Phi(V_j) / R0
    float* PW;          // sketch partials of W: (J*n_i2t) x (l1*l2)
    float* PV;          // sketch partials of the newest basis tensor
    float* SV;          // (m+1) x L sketched basis
    const float* SVx;   // Golub-Kahan: the other side's sketched basis
    double* dots;       // ntile[GRAM] x (m+2) x 2 partial inner products
    double* G;          // (m+1) x (m+1) Gram matrix of the sketched basis
    double* H;          // (m+1) x m Hessenberg, column-major
    double* R;          // m x m Givens-rotated H (upper triangular), column-major
    double* gv;         // cs[m], sn[m], g[m+1]
    float* coef;        // coefficients of the next multi-AXPY; coef[MMAX+1] = scale
    double* y;          // m
    int* state;         // NSTATE ints
    double* scal;       // NSCAL doubles
    // parameters
    double mu, delta, eta, stop_res, bd_tol;
};

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
// The workitem's index in its workgroup, read through an opaque register
// copy.  A stage body inlined into the loop of the persistent launch would
// otherwise have its per-lane index arithmetic hoisted out of the loop and
// kept in registers through every other stage (the stand-alone kernels
// compile to the same registers either way).
__device__ __forceinline__ int block_tid() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    __builtin_assume(t >= 0 && t < 1024);
    return t;
}

// Lane 0's value, known to the compiler to be the same in every lane.  A
// value that is uniform but comes from a vector memory load (a descriptor
// field, a problem's state word) otherwise lives in vector registers, and
// every buffer access whose resource is built from it is wrapped in a loop
// over the distinct values of the wave's lanes.
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int find_problem(const int* __restrict__ starts, int count, int b) {
    // largest p with starts[p] <= b (starts has count+1 entries, starts[0] = 0);
    // every lane of a wave asks for the same b, and the answer is made
    // wave-uniform
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (uniform_int(starts[mid]) <= b) lo = mid; else hi = mid - 1;
    }
    return uniform_int(lo);
}

// Operand order of the mode-1 sketch matrices for the MFMA contractions.
// The l1 x I1 matrix is cut into tiles of 16 rows (a) by K columns (i),
// K = 32 for bfloat16 (16x16x32 products) and 16 for float32 (16x16x4);
// tile (t, kb) is stored as 64 lanes x 16 bytes, lane m + 16 q holding row
// 16 t + m, columns kb K + q K/4 .. kb K + (q + 1) K/4 - 1, and tiles run
// kb fastest.  A wave then loads a whole tile with one contiguous 1 KB read.
// Rows past l1 and columns past I1 are zero.
constexpr int FRAG_K_BF16 = 32;
constexpr int FRAG_K_F32 = 16;
__host__ __device__ inline int frag_nkb(int I1, int k) { return (I1 + k - 1) / k; }
__host__ __device__ inline size_t frag_elems(int l1, int I1, int k) {
    return (size_t)((l1 + 15) / 16) * 16 * frag_nkb(I1, k) * k;
}
__host__ __device__ inline size_t frag_index(int a, int i, int nkb, int k) {
    const int per = k / 4, t = a >> 4, m = a & 15, kb = i / k, r = i % k;
    return (((size_t)t * nkb + kb) * 64 + m + 16 * (r / per)) * per + r % per;
}

// entries of the mode-1 part of the composition kernel's index space
// (rows padded to 16, columns to FRAG_K_BF16, so that padding is written)
__host__ __device__ inline size_t compose_mode1_entries(int l1, int I1) {
    return (size_t)((l1 + 15) / 16) * 16 * frag_nkb(I1, FRAG_K_BF16) * FRAG_K_BF16;
}

// Workgroups go to the chip's 8 XCDs round-robin by index, and each XCD has
// its own L2.  Renumbering so that XCD x takes the contiguous range of
// logical tiles [x q + min(x, r), ...) (q = total / 8, r = total % 8) keeps
// tiles of one problem, which read the same sketch matrices and overlapping
// halos, on one L2.  A bijection of [0, total).
__device__ __forceinline__ int xcd_tile(int b, int total) {
    const int q = total >> 3, r = total & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Identity sketch (unsketched global GMRES): tensor elements per Gram
// workgroup, and the workgroups of one problem
constexpr int FROB_CHUNK = 4096;
__host__ __device__ inline int frob_wgs(long long n) { return (int)((n + FROB_CHUNK - 1) / FROB_CHUNK); }

// Sketched-Gram workgroups whose pairs carry many partials (J channels x nt2
// column tiles above 48 per buffer) and few finished values (l3 <= 16) finish
// each pair with GRAM_SPL threads, each over a slice of the channels, and
// take GRAM_CH_SPLIT pairs.
constexpr int GRAM_SPL = 8;
constexpr int GRAM_CH_SPLIT = 256 / GRAM_SPL;
__host__ __device__ inline bool gram_split(int l3, int J, int nt2) { return J * nt2 > 48 && l3 <= 16; }

// (a, b) pairs of the sketch owned by one sketched-Gram workgroup
__host__ __device__ inline int gram_pairs_per_block(int l3, int J, int nt2) {
    if (gram_split(l3, J, nt2)) return GRAM_CH_SPLIT;
    int ch = 4096 / (l3 > 0 ? l3 : 1);
    if (ch > GRAM_CH) ch = GRAM_CH;
    if (ch < 1) ch = 1;
    return ch;
}

// bfloat16 values are handled as raw 16-bit patterns (round to nearest even)
__device__ __forceinline__ float bf2f(bf16_t u) { return __uint_as_float((unsigned)u << 16); }
// round to nearest even (v_cvt_pk_bf16_f32 on gfx950; NaN stays NaN)
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }

// Pointers read from descriptors are generic; loads through them become flat
// instructions (which also count against the LDS wait counter).  Tensor data
// always lives in device global memory, so cast to the global address space.
#define RTG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const RTG_GLOBAL T* gptr(const T* p) {
    return (const RTG_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ RTG_GLOBAL T* gptr_w(T* p) {
    return (RTG_GLOBAL T*)p;
}

// Mode-2 contraction of a column tile's mode-1 results (the second factor
// of the sketch, Sec. 3.1): for the stacked row tiles t < NRT,
//   P[a][b] = sum_k Ys[16 t + .][k] Om2x[b][i20 + k],
// with Om2 into P0 for t < RT and the composed Om2 A2 into P1 for t >= RT
// (P0, P1: l1 x l2 partials of this tile).  Ys holds 16 NRT rows of TC
// columns, row stride YP.  Wave w takes the pairs (t, column tile) with
// index w, w + 4, ...; the TC values of Om2x a lane needs for one column tile
// are loaded once per (column tile, matrix), all in flight together, by
// buffer loads that read zeros past l2 and past the tile's ncol columns.
// I2 l2 stays below 2^29 (sketch set-up limits), so 0x80000000 is past the
// buffer range.
template <int TC, int YP>
__device__ __forceinline__ void mode2_partials(const float* Ys, int wave, int lane, int NRT, int RT, int l1,
                                               int l2, int I2, int i20, int ncol, const float* om2,
                                               const float* om2t, float* P0, float* P1) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int m16 = lane & 15, kq = lane >> 4;
    const int RT2 = (l2 + 15) >> 4;
    const int obytes = l2 * I2 * 4;
    int key = -1;
    float Bv[TC / 4];
#pragma unroll
    for (int ks = 0; ks < TC / 4; ++ks) Bv[ks] = 0.f;
    for (int tt = wave; tt < NRT * RT2; tt += 4) {
        const int t = tt / RT2, rt2 = tt % RT2;
        const int half = t >= RT ? 1 : 0;
        const int bcol = 16 * rt2 + m16;
        if (2 * rt2 + half != key) {
            key = 2 * rt2 + half;
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(half ? om2t : om2), (short)0, obytes,
                                                              0x00020000);
#pragma unroll
            for (int ks = 0; ks < TC / 4; ++ks) {
                const int k = 4 * ks + kq;
                const unsigned off =
                    (bcol < l2 && k < ncol) ? (unsigned)(bcol * I2 + i20 + k) * 4u : 0x80000000u;
                Bv[ks] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
            }
        }
        // the transposed tile (Om2 rows as the A operand): lane (m16, kq)
        // then holds P[a = m16][b = 4 kq .. 4 kq + 3] of the 16 x 16 block,
        // four consecutive floats of one row -- one 16-byte store
        f4v pacc = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks)
            pacc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[ks], Ys[(16 * t + m16) * YP + 4 * ks + kq], pacc, 0, 0, 0);
        float* P = half ? P1 : P0;
        const int ar = 16 * (t - half * RT) + m16;
        const int b0 = 16 * rt2 + 4 * kq;
        if ((l2 & 3) == 0) {
            if (ar < l1 && b0 < l2) *gptr_w((f4v*)(P + (size_t)ar * l2 + b0)) = pacc;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (ar < l1 && b0 + i < l2) *gptr_w(P + (size_t)ar * l2 + b0 + i) = pacc[i];
        }
    }
}

// Fast path of the mode-2 contraction for 49 <= l2 <= 64 (four column tiles
// of Om2, one per wave): the wave's Om2 and Om2 A2 columns are requested
// together, before the mode-1 results reach LDS, so that one memory latency
// overlaps the barriers instead of two following them.
// B1 (the Om2 A2 columns) is loaded only for a dual sketch (NRT > RT): a
// sketch-only descriptor has no composed matrices.
template <int TC>
__device__ __forceinline__ void mode2_load4(int wave, int lane, int l2, int I2, int i20, int ncol, int NRT,
                                            int RT, const float* om2, const float* om2t, float (&B0)[TC / 4],
                                            float (&B1)[TC / 4]) {
    const int m16 = lane & 15, kq = lane >> 4;
    const int obytes = l2 * I2 * 4;
    const int bcol = 16 * wave + m16;
    const auto r0 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(om2), (short)0, obytes, 0x00020000);
#pragma unroll
    for (int ks = 0; ks < TC / 4; ++ks) {
        const int k = 4 * ks + kq;
        const unsigned off = (bcol < l2 && k < ncol) ? (unsigned)(bcol * I2 + i20 + k) * 4u : 0x80000000u;
        B0[ks] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r0, off, 0, 0));
        B1[ks] = 0.f;
    }
    if (NRT > RT) {
        const auto r1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(om2t), (short)0, obytes, 0x00020000);
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks) {
            const int k = 4 * ks + kq;
            const unsigned off = (bcol < l2 && k < ncol) ? (unsigned)(bcol * I2 + i20 + k) * 4u : 0x80000000u;
            B1[ks] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r1, off, 0, 0));
        }
    }
}

template <int TC, int YP>
__device__ __forceinline__ void mode2_partials4(const float* Ys, int wave, int lane, int NRT, int RT, int l1, int l2,
                                                const float (&B0)[TC / 4], const float (&B1)[TC / 4], float* P0,
                                                float* P1) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int m16 = lane & 15, kq = lane >> 4;
    const int b0 = 16 * wave + 4 * kq;
    auto one = [&](int t, const float (&Bv)[TC / 4], float* P, int ar) {
        f4v pacc = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks)
            pacc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[ks], Ys[(16 * t + m16) * YP + 4 * ks + kq], pacc, 0, 0, 0);
        if ((l2 & 3) == 0) {
            if (ar < l1 && b0 < l2) *gptr_w((f4v*)(P + (size_t)ar * l2 + b0)) = pacc;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (ar < l1 && b0 + i < l2) *gptr_w(P + (size_t)ar * l2 + b0 + i) = pacc[i];
        }
    };
    for (int t = 0; t < RT; ++t) one(t, B0, P0, 16 * t + m16);
    if (NRT > RT)
        for (int t = 0; t < RT; ++t) one(RT + t, B1, P1, 16 * t + m16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace rtg

// ---------------------------------------------------------------------------
// host-side launchers (one per translation unit)
// ---------------------------------------------------------------------------
namespace rtg {
int phi_jt(int max_j);
int phi_tiles(int I1, int I2, int J, int jt);
hipError_t launch_phi(const Desc* d, const int* starts, int count, int total_tiles,
                      int src_sel, int src_index, int rmax, int jt, int bf16_in, hipStream_t s,
                      int stencil = 0, int slab = 0, int toeplitz = 0);
hipError_t launch_phi_single(int I1, int I2, int J, int r1, int r2, int rB, const float* a1,
                             const float* a2, const float* bb, const float* st, const float* taps,
                             const void* src, int bf16_in, const float* C, float* dst, hipStream_t s);
hipError_t launch_tile(const Desc* d, const int* starts, int count, int total_tiles,
                       int mode, int nterms, int dst_index, int basis_bf16, int src_bf16,
                       int l1max, hipStream_t s, int first_term = 0, int rows = 2, int sketch_bf16 = 0);
// rows (tile and step kernels): 16-row sketch tiles per wave, 2 where the
// stacked sketch rows fit (the default), or 4
hipError_t launch_step(const Desc* d, const int* starts, int count, int total_tiles, int j, int rmax,
                       int basis_bf16, int l1max, int toeplitz, hipStream_t s, int rows = 2);
hipError_t launch_gram(const Desc* d, const int* starts, int count, int total_tiles,
                       int mode, int j, float* sketch_out, hipStream_t s, int unsketched = 0);
hipError_t launch_solve(const Desc* d, int count, int mmax, hipStream_t s);
// sched (may be null): the persistent launch's words, zeroed by block 0
hipError_t launch_init(const Desc* d, int count, hipStream_t s, int cycle = 0, int* sched = nullptr);
hipError_t launch_compose(const Desc* d, int count, int max_entries, hipStream_t s);
hipError_t launch_finish_arnoldi(const Desc* d, double* H, double* beta, int* m_done,
                                 int m, hipStream_t s);

// The persistent launch of a batch's Arnoldi process: its scheduling words
// (next task, error, workgroups that have left) and arguments.
// (one task counter per XCD queue, each on its own 128-byte line)
enum { SCH_ERROR = 0, SCH_EXITED = 1, SCH_QUEUE = 32, SCH_QSTRIDE = 32, SCH_WORDS = SCH_QUEUE + 8 * SCH_QSTRIDE };
struct PersistArgs {
    const Desc* descs;
    const int* starts[NKIND];   // prefix tables of the problems' tiles per kernel kind
    int count;
    int qfirst[NKIND][9];       // per kernel kind, the first tile of each XCD queue's problems (and the total)
    int steps;                  // Arnoldi steps (the largest m)
    int full;                   // steps that form V_{j+1} (the operator and tile stages)
    int any_x0;                 // the operator on X0 comes first
    int cycle;                  // restart cycle (the start stage's argument)
    int* sched;                 // SCH_WORDS ints, zeroed before the launch
    int wait_limit;             // polls before a wait gives up
};
hipError_t launch_persist(const PersistArgs& a, int rmax, int toeplitz, int sketch_bf16, hipStream_t s);

// k_tile modes
// (TM_GKNEW: a new Golub-Kahan basis tensor from W and the terms
// [first_term, nterms) of this side's basis)
// (TM_SKETCH_W: the sketch of the stored W, for operators without composed
// sketch matrices)
// (TM_NEWV1: V_1 = R0 of a bfloat16 basis stored unnormalised: where X0 is
// given, the operator kernel (PS_X0_V1) has stored R0 = C - Phi(X0) in
// bfloat16 as V_1 already and the pass only sketches it; otherwise R0 = C is
// rounded, stored and sketched as TM_NEWV does)
enum TileMode { TM_NEWV = 1, TM_ASSEMBLE = 2, TM_SKETCH_SRC = 3, TM_GKNEW = 4, TM_SKETCH_W = 5, TM_NEWV1 = 6 };
// k_phi source selection (PS_X0_V1: R0 = C - Phi(X0) rounded to bfloat16
// into the basis' first slot)
enum PhiSrc { PS_BASIS = 0, PS_X0 = 1, PS_X0_V1 = 2 };
// k_gram modes
// (GM_GK: one Golub-Kahan half-step, the sketched norm of the next tensor)
enum GramMode { GM_START = 0, GM_STEP = 1, GM_SKETCH_OUT = 2, GM_GK = 3 };
}  // namespace rtg
