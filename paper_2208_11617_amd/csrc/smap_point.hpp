// smap_point.hpp -- per-element kernels MAP, ACCUM, HITS and HASH (uint32).
//
// One workgroup of 256 threads processes one tile of rho^m elements (the
// test kernels of Section 5.1, Table tab:tests; HITS and HASH added).  Lanes
// run along x_1, so a wave touches whole rho-element row segments.  The tile
// comes from the H decode (one 1-D grid over the fused native + shell
// pieces) or from the BB grid coordinates.  Only tiles that cross the
// simplex boundary filter their elements (sum x <= n); tiles fully inside
// skip the test, and BB tiles fully outside exit before touching memory.
//
// Element offsets inside a tile are separable: for the tile-local index
// li = tid + 256 e (tid < 256) every coordinate bit-field of li is the sum
// of its field in tid and its field in 256 e, so offset(li) = offset(tid) +
// offset(256 e), the second term being a compile-time multiple of the
// strides (scalar).  Per element the lane does one add and, in boundary
// tiles only, one compare.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_decode.hpp"

namespace smap {

enum Op { OP_MAP = 0, OP_ACCUM = 1, OP_HITS = 2, OP_HASH = 3, OP_CA2 = 4, OP_CA3 = 5 };

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int ipowc(int b, int e) { return e == 0 ? 1 : b * ipowc(b, e - 1); }

// hash32: FNV-1a over the 32-bit words x_1..x_m, then MurmurHash3's fmix32.
template <int M>
__device__ __forceinline__ uint32_t hash32_words(const int32_t *x)
{
    uint32_t h = 0x811C9DC5u;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        h ^= (uint32_t)x[k];
        h *= 0x01000193u;
    }
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Tile coordinates of this workgroup, or false if it has none.
template <int M, bool BB>
__device__ __forceinline__ bool wg_tile(const Plan &P, int32_t *t)
{
    if (BB) {
        decode_bb(P, blockIdx.x, blockIdx.y, blockIdx.z, t);
        return true;
    }
    return decode_h<M>(P, blockIdx.x, t);
}

template <int M, int RHO, int OP, bool BB>
__global__ __launch_bounds__(256) void k_point(const Plan P, const uint32_t *in, uint32_t *out)
{
    constexpr int LR = ilog2c(RHO);
    constexpr int NE = ipowc(RHO, M);
    constexpr int E = NE / 256;
    static_assert(NE % 256 == 0, "tile must hold a multiple of 256 elements");

    int32_t t[4] = {0, 0, 0, 0};
    if (!wg_tile<M, BB>(P, t)) return;
    int32_t x0[M];
    int32_t s0 = 0;
    int64_t base = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        x0[k] = t[k] * RHO;
        s0 += x0[k];
        base += (int64_t)x0[k] * P.stride[k];
    }
    const int32_t n = P.n;
    if (s0 > n) return;                               // BB tile outside the simplex
    const bool full = s0 + M * (RHO - 1) <= n;

    // per-thread part of the tile-local coordinates and offset
    const uint32_t tid = threadIdx.x;
    int32_t lt[M];
    int32_t st = 0;
    uint32_t ot = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        lt[k] = (int32_t)((tid >> (k * LR)) & (RHO - 1));
        st += lt[k];
        ot += (uint32_t)lt[k] * (uint32_t)P.stride[k];
    }
    const uint32_t *pin = in + base;
    uint32_t *pout = out + base;

#pragma unroll
    for (int e = 0; e < E; ++e) {
        // the per-iteration part: fields of 256 e (compile-time bit fields)
        const uint32_t hi = (uint32_t)e * 256u;
        int32_t le[M];
        int32_t se = 0;
        uint32_t oe = 0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            le[k] = (int32_t)((hi >> (k * LR)) & (RHO - 1));
            se += le[k];
            oe += (uint32_t)le[k] * (uint32_t)P.stride[k];
        }
        if (!full && s0 + st + se > n) continue;
        const uint32_t off = ot + oe;
        if (OP == OP_MAP) {
            asm volatile("" ::"v"(off));                 // keep the mapping, drop nothing
        } else if (OP == OP_ACCUM) {
            pout[off] = pin[off] + 1u;
        } else if (OP == OP_HITS) {
            atomicAdd(pout + off, 1u);
        } else if (OP == OP_HASH) {
            int32_t x[M];
#pragma unroll
            for (int k = 0; k < M; ++k) x[k] = x0[k] + lt[k] + le[k];
            pout[off] = hash32_words<M>(x);
        }
    }
}

}  // namespace smap
