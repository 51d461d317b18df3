// Tile kernel (the stage itself is tile_task in tile_body.h).
#include "tile_body.h"

namespace rtg {

template <bool BB, bool MB, bool SPLIT, int RPW>
__global__ void __launch_bounds__(256) k_tile(const Desc* __restrict__ descs,
                                              const int* __restrict__ starts, int count,
                                              int mode, int nterms_arg, int dst_index, int t0) {
    __shared__ TileShared<MB, SPLIT, RPW> sh;
    tile_task<BB, MB, SPLIT, RPW>(descs, starts, count, mode, nterms_arg, dst_index, t0, blockIdx.x, sh);
}

hipError_t launch_tile(const Desc* d, const int* starts, int count, int total_tiles, int mode,
                       int nterms, int dst_index, int basis_bf16, int src_bf16, int l1max, hipStream_t s,
                       int first_term, int rows, int sketch_bf16) {
#define RTG_TILE(BBV, MBV, SPV, RPV)                                                              \
    hipLaunchKernelGGL((k_tile<BBV, MBV, SPV, RPV>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, \
                       mode, nterms, dst_index, first_term)
    const int rtiles = ((l1max + 15) / 16) * ((mode == TM_NEWV || mode == TM_GKNEW || mode == TM_NEWV1) ? 2 : 1);
    const bool small = rtiles <= 8 && rows != 4;
    const bool split = (mode == TM_SKETCH_SRC || mode == TM_SKETCH_W) && !src_bf16;
    if (basis_bf16) {
        if (split) { if (small) RTG_TILE(true, true, true, 2); else RTG_TILE(true, true, true, 4); }
        else { if (small) RTG_TILE(true, true, false, 2); else RTG_TILE(true, true, false, 4); }
    } else if (sketch_bf16) {
        // float32 basis with bfloat16 products: sources that are not a basis
        // tensor (R0, W) keep the two-plane split, new basis tensors one plane
        if (split) { if (small) RTG_TILE(false, true, true, 2); else RTG_TILE(false, true, true, 4); }
        else { if (small) RTG_TILE(false, true, false, 2); else RTG_TILE(false, true, false, 4); }
    } else {
        if (small) RTG_TILE(false, false, false, 2); else RTG_TILE(false, false, false, 4);
    }
#undef RTG_TILE
    return hipGetLastError();
}

}  // namespace rtg
