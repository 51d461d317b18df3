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
enum { ST_ACTIVE = 0, ST_MEFF = 1, ST_FLAGS = 2, ST_COUNTER = 3, NSTATE = 16 };
// scal[] slots (double)
enum { SC_BETA = 0, SC_MU = 1, SC_RESPROJ = 2, SC_RESLS = 3, SC_RHO = 4, NSCAL = 16 };

struct Desc {
    // sizes
    int I1, I2, J;
    int l1, l2, l3;
    int r1, r2, rB;
    int m;              // max steps for this problem
    int bf16;           // basis stored as bfloat16
    int has_om3;        // Om3 given (else identity, l3 == J)
    int n_i2t;          // ceil(I2 / TILE_TC)
    int ntile[NKIND];   // tiles of this problem per kernel kind
    int mu_fixed;       // 1: mu given, 0: discrepancy principle
    int keep_last;      // form V_{m+1} after the last step (Arnoldi-only calls)
    long long n;        // I1*I2*J
    long long L;        // l1*l2*l3
    // operator / sketch (device)
    const float* a1;
    const float* a2;
    const float* bb;
    const float* a1t;             // bands transposed: a1t[(r1 + dd) I1 + i] = a1[i (2 r1 + 1) + r1 + dd]
    const float* a2t;
    const float* a1p[3];          // A1 band rows zero-padded to the tiers R = 4, 8, 12 (row stride 2R+1 rounded up to 4)
    const float* om1;
    const bf16_t* om1h;           // bfloat16 copy of Om1
    const float* om2;
    const float* om3;             // nullptr => identity
    // sketch of Phi(X) as a sketch of X (mode products compose, eq. (2)):
    // Om1 A1 (float32, and bfloat16 high/low planes), Om2 A2, Om3 B^T (l3 x J)
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
__device__ __forceinline__ int find_problem(const int* __restrict__ starts, int count, int b) {
    // largest p with starts[p] <= b (starts has count+1 entries, starts[0] = 0)
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// (a, b) pairs of the sketch owned by one sketched-Gram workgroup
__host__ __device__ inline int gram_pairs_per_block(int l3) {
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
                      int src_sel, int src_index, int rmax, int jt, int bf16_in, hipStream_t s);
hipError_t launch_phi_single(int I1, int I2, int J, int r1, int r2, int rB, const float* a1,
                             const float* a2, const float* bb, const void* src, int bf16_in,
                             const float* C, float* dst, hipStream_t s);
hipError_t launch_tile(const Desc* d, const int* starts, int count, int total_tiles,
                       int mode, int nterms, int dst_index, int basis_bf16, int src_bf16,
                       int l1max, hipStream_t s);
hipError_t launch_step(const Desc* d, const int* starts, int count, int total_tiles, int j, int rmax,
                       int basis_bf16, int l1max, hipStream_t s);
hipError_t launch_gram(const Desc* d, const int* starts, int count, int total_tiles,
                       int mode, int j, float* sketch_out, hipStream_t s);
hipError_t launch_solve(const Desc* d, int count, int mmax, hipStream_t s);
hipError_t launch_init(const Desc* d, int count, hipStream_t s);
hipError_t launch_compose(const Desc* d, int count, int max_entries, hipStream_t s);
hipError_t launch_finish_arnoldi(const Desc* d, double* H, double* beta, int* m_done,
                                 int m, hipStream_t s);

// k_tile modes
enum TileMode { TM_NEWV = 1, TM_ASSEMBLE = 2, TM_SKETCH_SRC = 3 };
// k_phi source selection
enum PhiSrc { PS_BASIS = 0, PS_X0 = 1 };
// k_gram modes
enum GramMode { GM_START = 0, GM_STEP = 1, GM_SKETCH_OUT = 2 };
}  // namespace rtg
