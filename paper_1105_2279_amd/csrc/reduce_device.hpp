// Deterministic FP64 reduction of per-group partial sums.  The same code
// runs as two kernels (single-lattice calls) or inside one block (the
// batched kernel), so both give bit-identical results.
#pragma once

#include "qdpx_impl.hpp"
#include "su3_device.hpp"

namespace qdpx {

constexpr int kFinChunk = 16;
constexpr int kFinPerBlock = kReduceBlock * kFinChunk;

// Stage A for chunk b of n values: thread t adds its 16 consecutive values
// in order, then a fixed block tree.  Result valid in thread 0.
__device__ __forceinline__ double fin_stage_a(const double *__restrict__ p, int n, int b, double *lds) {
    const int base = b * kFinPerBlock + (int)threadIdx.x * kFinChunk;
    const auto *gp = gptr<double>(p);  // partials always live in global memory
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kFinChunk; ++k)
        if (base + k < n) v += gp[base + k];
    return block_sum<kReduceBlock / 64>(v, lds);
}

// Stage B over nb stage-A values: strided per-thread sums, then the tree.
__device__ __forceinline__ double fin_stage_b(const double *p, int nb, double *lds) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kReduceBlock) v += p[i];
    return block_sum<kReduceBlock / 64>(v, lds);
}

// mode 0: out[0] = r[0]; mode 1: plaquette triple from spatial r[0] and temporal r[1].
__device__ __forceinline__ void fin_write(const double r[2], int mode, double volume, double *out) {
    if (mode == 0) {
        out[0] = r[0];
    } else {
        out[0] = (r[0] + r[1]) / (18.0 * volume);
        out[1] = r[0] / (9.0 * volume);
        out[2] = r[1] / (9.0 * volume);
    }
}

}  // namespace qdpx
