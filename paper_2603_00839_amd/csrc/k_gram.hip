// Sketched-Gram kernel (the stage itself is gram_task in gram_body.h).
#include "gram_body.h"

namespace rtg {

template <bool FROB>
__global__ void __launch_bounds__(256) k_gram(const Desc* __restrict__ descs,
                                              const int* __restrict__ starts, int count, int mode,
                                              int j, float* sketch_out) {
    __shared__ GramSmem sm;
    gram_task<FROB>(descs, starts, count, mode, j, sketch_out, blockIdx.x, sm);
}

hipError_t launch_gram(const Desc* d, const int* starts, int count, int total_tiles, int mode, int j,
                       float* sketch_out, hipStream_t s, int unsketched) {
    if (unsketched)
        hipLaunchKernelGGL(k_gram<true>, dim3(total_tiles), dim3(256), 0, s, d, starts, count, mode, j, sketch_out);
    else
        hipLaunchKernelGGL(k_gram<false>, dim3(total_tiles), dim3(256), 0, s, d, starts, count, mode, j, sketch_out);
    return hipGetLastError();
}

}  // namespace rtg
