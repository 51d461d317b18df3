// Operator kernels (the tile itself is phi_tile in phi_body.h).
#include "phi_body.h"

namespace rtg {

template <int R, bool BF16IN, int JT, bool ST, int SL, bool TP>
__global__ void __launch_bounds__(256) k_phi_single(PhiArgs a) {
    __shared__ __attribute__((aligned(16))) float smem[PhiLayout<R, JT, SL>::FLOATS];
    phi_tile<R, BF16IN, JT, ST, SL, TP>(a, xcd_remap(blockIdx.x, gridDim.x), smem);
}

template <int R, bool BF16IN, int JT, bool ST, int SL, bool TP>
__global__ void __launch_bounds__(256) k_phi_batched(const Desc* __restrict__ descs,
                                                     const int* __restrict__ starts, int count,
                                                     int src_sel, int src_index) {
    __shared__ __attribute__((aligned(16))) float smem[PhiLayout<R, JT, SL>::FLOATS];
    phi_batched_task<R, BF16IN, JT, ST, SL, TP>(descs, starts, count, src_sel, src_index,
                                                xcd_remap(blockIdx.x, gridDim.x), smem);
}

static int phi_tier(int r) { return r <= 4 ? 4 : (r <= 8 ? 8 : 12); }

int phi_jt(int max_j) { return max_j <= 4 ? 4 : 8; }

int phi_tiles(int I1, int I2, int J, int jt) {
    return ((I1 + PHI_T1 - 1) / PHI_T1) * ((I2 + PHI_T2 - 1) / PHI_T2) * ((J + jt - 1) / jt);
}

hipError_t launch_phi_single(int I1, int I2, int J, int r1, int r2, int rB, const float* a1,
                             const float* a2, const float* bb, const float* st, const float* taps,
                             const void* src, int bf16_in, const float* C, float* dst, hipStream_t s) {
    PhiArgs a{I1, I2, J, r1, r2, rB, a1, a2, bb, src, C, dst, st, taps};
    const int jt = phi_jt(J);
    const int tiles = phi_tiles(I1, I2, J, jt);
    const int tier = phi_tier(r1 > r2 ? r1 : r2);
    // 16-byte slab loads need 32-bit byte offsets into the float32 input;
    // asynchronous ones (general PSF) every channel in one tile (J <= 3);
    // Toeplitz taps in registers with the 16-byte staging
    const bool vec = !bf16_in && (size_t)I1 * I2 * J * 4 <= 0x7FFFFFFFull;
    const bool dma = vec && st != nullptr && J <= 3;
    const bool tp = vec && st == nullptr && taps != nullptr;
#define RTG_PHI_SINGLE_K(RR, BB, JJ, SS, LL, TT) \
    hipLaunchKernelGGL((k_phi_single<RR, BB, JJ, SS, LL, TT>), dim3(tiles), dim3(256), 0, s, a);
#define RTG_PHI_SINGLE_S(RR, JJ, SS)                                                     \
    if (bf16_in) { RTG_PHI_SINGLE_K(RR, true, JJ, SS, SL_SCALAR, false) }               \
    else if (dma && JJ == 4) { RTG_PHI_SINGLE_K(RR, false, 4, SS, SL_DMA, false) }     \
    else if (tp && !SS) { RTG_PHI_SINGLE_K(RR, false, JJ, false, SL_VEC, true) }        \
    else if (vec) { RTG_PHI_SINGLE_K(RR, false, JJ, SS, SL_VEC, false) }                \
    else { RTG_PHI_SINGLE_K(RR, false, JJ, SS, SL_SCALAR, false) }
#define RTG_PHI_SINGLE(RR, JJ) if (st) { RTG_PHI_SINGLE_S(RR, JJ, true) } else { RTG_PHI_SINGLE_S(RR, JJ, false) }
#define RTG_PHI_SINGLE_J(RR) if (jt == 4) { RTG_PHI_SINGLE(RR, 4) } else { RTG_PHI_SINGLE(RR, 8) }
    if (tier == 4) { RTG_PHI_SINGLE_J(4) } else if (tier == 8) { RTG_PHI_SINGLE_J(8) } else { RTG_PHI_SINGLE_J(12) }
#undef RTG_PHI_SINGLE_J
#undef RTG_PHI_SINGLE
#undef RTG_PHI_SINGLE_S
#undef RTG_PHI_SINGLE_K
    return hipGetLastError();
}

// slab: 0 = single-word staging only, 1 = 16-byte loads possible (float32
// inputs below 2^31 bytes), 2 = also asynchronous loads (and J <= 3);
// toeplitz: every problem's bands are Toeplitz (taps in registers)
hipError_t launch_phi(const Desc* d, const int* starts, int count, int total_tiles, int src_sel,
                      int src_index, int rmax, int jt, int bf16_in, hipStream_t s, int stencil, int slab,
                      int toeplitz) {
    const int tier = phi_tier(rmax);
    const bool vec = !bf16_in && slab >= 1;
    const bool dma = vec && stencil && slab >= 2;
    const bool tp = vec && !stencil && toeplitz;
#define RTG_PHI_BATCH_K(RR, BB, JJ, SS, LL, TT)                                                                      \
    hipLaunchKernelGGL((k_phi_batched<RR, BB, JJ, SS, LL, TT>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, \
                       src_sel, src_index);
#define RTG_PHI_BATCH_S(RR, JJ, SS)                                                   \
    if (bf16_in) { RTG_PHI_BATCH_K(RR, true, JJ, SS, SL_SCALAR, false) }             \
    else if (dma && JJ == 4) { RTG_PHI_BATCH_K(RR, false, 4, SS, SL_DMA, false) }   \
    else if (tp && !SS) { RTG_PHI_BATCH_K(RR, false, JJ, false, SL_VEC, true) }      \
    else if (vec) { RTG_PHI_BATCH_K(RR, false, JJ, SS, SL_VEC, false) }              \
    else { RTG_PHI_BATCH_K(RR, false, JJ, SS, SL_SCALAR, false) }
#define RTG_PHI_BATCH(RR, JJ) if (stencil) { RTG_PHI_BATCH_S(RR, JJ, true) } else { RTG_PHI_BATCH_S(RR, JJ, false) }
#define RTG_PHI_BATCH_J(RR) if (jt == 4) { RTG_PHI_BATCH(RR, 4) } else { RTG_PHI_BATCH(RR, 8) }
    if (tier == 4) { RTG_PHI_BATCH_J(4) } else if (tier == 8) { RTG_PHI_BATCH_J(8) } else { RTG_PHI_BATCH_J(12) }
#undef RTG_PHI_BATCH_J
#undef RTG_PHI_BATCH
#undef RTG_PHI_BATCH_S
#undef RTG_PHI_BATCH_K
    return hipGetLastError();
}

}  // namespace rtg
