// Paired launches: the array and its mirror run the same kernel of a fused
// window in one launch.  The grid's y index picks the argument set (0: the
// array, 1: the mirror); blockIdx.x, gridDim.x and the block are those of a
// single launch, so each kernel body runs unchanged.  Each Op names its
// argument block (Args) and its body (run).
#pragma once

#include "common.h"

namespace gpma_dev {

template <class Op, int TPB>
__global__ void __launch_bounds__(TPB) k_pair(typename Op::Args a0, typename Op::Args a1) {
    Op::run(blockIdx.y ? a1 : a0);
}

}  // namespace gpma_dev

namespace gpma_host {

template <class Op, int TPB>
inline void launch_pair(uint32_t gx, const typename Op::Args &a0, const typename Op::Args &a1, hipStream_t s) {
    hipLaunchKernelGGL((gpma_dev::k_pair<Op, TPB>), dim3(gx, 2), dim3(TPB), 0, s, a0, a1);
}

}  // namespace gpma_host
