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

namespace smap {

// ---- persistent work-queue launch -----------------------------------------
//
// One launch for a mixed batch of CA2 and CA3 jobs.  The grid is sized to
// what the device holds at once (not to the work); each workgroup loops,
// claiming the next work unit with an atomic add on a head counter in
// device memory, until the head passes the tail (the total unit count,
// fixed at launch).  Units are the jobs' H-mapped tiles (times sub-blocks),
// concatenated job after job, so a workgroup maps a claimed unit to its job
// by the same binary search as the batched kernels.  Every workgroup ends:
// the head only grows, and a claim at or past the tail exits the loop.

enum QueueKind : uint32_t { kQueueCa2 = 0, kQueueCa3 = 1, kQueueCa2Small = 2, kQueueCa3Small = 3 };

struct QueueJob {
    Plan P;
    const uint8_t *in;
    uint8_t *out;
    uint32_t kind;        // QueueKind
    uint32_t reserved;
};

// Tile shapes of the queue kernel (256 threads for both classes): CA2
// rho 256 with one workgroup per tile; CA3 rho 64, 64 rows by one row per
// lane, 16 planes per sub-block, 4 sub-blocks per tile.
constexpr int kQueueThreads = 256;
constexpr int kQueueCa2Rho = 256, kQueueCa2W = 4, kQueueCa2R = 16, kQueueCa2D = 2;
constexpr int kQueueCa3Rho = 64, kQueueCa3Ry = 64, kQueueCa3Rz = 16, kQueueCa3Rl = 1;
// Jobs with n below this are small: one work unit each, stepped cell by cell.
constexpr int32_t kQueueSmallN = 15;

// One automaton step of a whole small job (n < 15: rows shorter than the
// 16-byte accesses of the tiled bodies) by one workgroup, a cell per
// thread: the clipped neighbourhood is counted with every neighbour
// checked against the simplex (B3/S23 for m = 2, B6/S567 for m = 3).
template <int M>
__device__ __forceinline__ void queue_small_step(const Plan &P, const uint8_t *__restrict__ in,
                                                 uint8_t *__restrict__ out)
{
    const int32_t n = P.n, w = n + 1;
    const int32_t cells = M == 2 ? w * w : w * w * w;
    for (int32_t c = (int32_t)threadIdx.x; c < cells; c += kQueueThreads) {
        const int32_t x = c % w, y = (c / w) % w, z = M == 3 ? c / (w * w) : 0;
        if (x + y + z > n) continue;
        uint32_t cnt = 0;
        for (int32_t dz = (M == 3 ? -1 : 0); dz <= (M == 3 ? 1 : 0); ++dz)
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    const int32_t X = x + dx, Y = y + dy, Z = z + dz;
                    if ((dx | dy | dz) == 0 || X < 0 || Y < 0 || Z < 0 || X + Y + Z > n) continue;
                    cnt += in[(Z * w + Y) * w + X] == 1 ? 1u : 0u;
                }
        const bool alive = in[c] == 1;
        const bool next = M == 2 ? (cnt == 3 || (alive && cnt == 2))
                                 : (alive ? (cnt >= 5 && cnt <= 7) : cnt == 6);
        out[c] = next ? 1 : 0;
    }
}

// Clears `count` words (a graph's head counter before each replay: a kernel
// node rather than a memset node).
__global__ __launch_bounds__(64) void k_zero_words(uint32_t *__restrict__ p, uint32_t count)
{
    for (uint32_t i = threadIdx.x; i < count; i += 64) p[i] = 0u;
}

__global__ __launch_bounds__(kQueueThreads) void k_queue(uint32_t *__restrict__ head,
                                                         const uint32_t *__restrict__ start,
                                                         const QueueJob *__restrict__ jobs, uint32_t njobs,
                                                         uint32_t total)
{
    constexpr uint32_t SUB2 = Ca2Walk<kQueueCa2Rho, kQueueCa2W, kQueueCa2R>::SUB;
    constexpr uint32_t SUB3 = Ca3Walk<kQueueCa3Rho, kQueueCa3Ry, kQueueCa3Rz, kQueueCa3Rl>::SUB;
    static_assert(64 * kQueueCa2W == kQueueThreads &&
                  Ca3Walk<kQueueCa3Rho, kQueueCa3Ry, kQueueCa3Rz, kQueueCa3Rl>::NT == kQueueThreads,
                  "queue tile shapes must use the whole workgroup");
    __shared__ uint32_t claim;
    for (;;) {
        if (threadIdx.x == 0) claim = atomicAdd(head, 1u);
        lds_barrier();
        const uint32_t u = __builtin_amdgcn_readfirstlane(claim);
        lds_barrier();     // every wave has read `claim` before the next claim overwrites it
        if (u >= total) return;
        const uint32_t j = batch_find(start, njobs, u);
        const uint32_t local = u - start[j];
        const QueueJob &J = jobs[j];
        const uint32_t kind = J.kind;   // uniform: every wave takes the same branch
        int32_t t[4] = {0, 0, 0, 0};
        if (kind == kQueueCa2) {
            if (decode_h<2>(J.P, local / SUB2, t))
                ca2_tile<kQueueCa2Rho, kQueueCa2W, kQueueCa2R, kQueueCa2D, false>(J.P, J.in, J.out, t,
                                                                                local % SUB2);
        } else if (kind == kQueueCa3) {
            // ca3_tile has barriers; the whole workgroup runs it
            if (decode_h<3>(J.P, local / SUB3, t))
                ca3_tile<kQueueCa3Rho, kQueueCa3Ry, kQueueCa3Rz, kQueueCa3Rl, false>(J.P, J.in, J.out, t,
                                                                                   local % SUB3);
        } else if (kind == kQueueCa2Small) {
            queue_small_step<2>(J.P, J.in, J.out);
        } else {
            queue_small_step<3>(J.P, J.in, J.out);
        }
    }
}

}  // namespace smap
