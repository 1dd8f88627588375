// smap_batch.hpp -- batched automaton steps: many jobs, one launch per class.
//
// The H-mapped workgroup ranges of the jobs are concatenated: job j owns the
// workgroups [start[j], start[j+1]) of the launch.  A workgroup finds its
// job by a binary search over `start` (wave-uniform, scalar loads), then
// decodes its tile with the job's own plan and runs the same tile body as
// the single-job kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_ca3.hpp"
#include "smap_decode.hpp"

namespace smap {

// One job of a batched launch, as the kernels read it from device memory.
struct BatchJob {
    Plan P;               // the job's H plan (its grid fields are unused)
    const uint8_t *in;
    uint8_t *out;
};

// Largest j in [0, njobs) with start[j] <= g, given start[0] = 0 <= g.
__device__ __forceinline__ uint32_t batch_find(const uint32_t *__restrict__ start, uint32_t njobs,
                                               uint32_t g)
{
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// CA2 jobs: SUB workgroups per tile of each job (its H grid times SUB).
template <int RHO, int W, int R, int D, bool SAFE>
__global__ __launch_bounds__(64 * W) void k_ca2_batch(const uint32_t *__restrict__ start,
                                                      const BatchJob *__restrict__ jobs, uint32_t njobs,
                                                      uint32_t nwg)
{
    constexpr int SUB = Ca2Walk<RHO, W, R>::SUB;
    const uint32_t g = xcd_remap(blockIdx.x, nwg);
    const uint32_t j = batch_find(start, njobs, g);
    const uint32_t local = g - start[j];
    const BatchJob &J = jobs[j];
    int32_t t[4] = {0, 0, 0, 0};
    if (!decode_h<2>(J.P, local / SUB, t)) return;
    ca2_tile<RHO, W, R, D, SAFE>(J.P, J.in, J.out, t, local % SUB);
}

// CA3 jobs: SUB workgroups per tile, tile-major within a job.
template <int RHO, int RY, int RZ, int RL, bool SAFE>
__global__ __launch_bounds__((RHO / 16) * (RY / RL)) void k_ca3_batch(const uint32_t *__restrict__ start,
                                                                      const BatchJob *__restrict__ jobs,
                                                                      uint32_t njobs, uint32_t nwg)
{
    constexpr int SUB = Ca3Walk<RHO, RY, RZ, RL>::SUB;
    const uint32_t g = blockIdx.x;
    const uint32_t j = batch_find(start, njobs, g);
    const uint32_t local = g - start[j];
    const BatchJob &J = jobs[j];
    int32_t t[4] = {0, 0, 0, 0};
    if (!decode_h<3>(J.P, local / SUB, t)) return;
    ca3_tile<RHO, RY, RZ, RL, SAFE>(J.P, J.in, J.out, t, local % SUB);
}

}  // namespace smap
