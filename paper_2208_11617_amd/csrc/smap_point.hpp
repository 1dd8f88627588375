// smap_point.hpp -- per-element kernels MAP, ACCUM, HITS, HASH (uint32) and
// EDM (float32).
//
// The test kernels of Section 5.1, Table tab:tests, plus HITS and HASH.  EDM
// (2-D only) stores at element (x_1, x_2) the distance between points
// i = x_1 and j = n - x_2 of a set of n+1 points in R^3 (x_1 + x_2 <= n is
// i <= j), in float32: three differences, a sum of squares, sqrtf.
// The tile comes from the H decode (one 1-D grid over the fused native +
// shell pieces) or from the BB grid coordinates; BB tiles fully outside the
// simplex exit before touching memory.
//
// Rows of the box are unaligned for a general n (pitch n+1 elements); gfx9
// global memory accepts unaligned 16-byte accesses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_decode.hpp"

namespace smap {

enum Op { OP_MAP = 0, OP_ACCUM = 1, OP_HITS = 2, OP_HASH = 3, OP_CA2 = 4, OP_CA3 = 5, OP_EDM = 6 };

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int ipowc(int b, int e) { return e == 0 ? 1 : b * ipowc(b, e - 1); }

// hash32: FNV-1a over the 32-bit words x_1..x_m, then MurmurHash3's fmix32.
// hash32_state<K0, K1>(h, x) runs the FNV-1a steps of words K0..K1-1 from
// state h (the offset basis 0x811C9DC5 before the first word), so a state
// over leading words that several elements share can be computed once.
template <int K0, int K1>
__device__ __forceinline__ uint32_t hash32_state(uint32_t h, const int32_t *x)
{
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        h ^= (uint32_t)x[k];
        h *= 0x01000193u;
    }
    return h;
}

__device__ __forceinline__ uint32_t hash32_fmix(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

template <int M>
__device__ __forceinline__ uint32_t hash32_words(const int32_t *x)
{
    return hash32_fmix(hash32_state<0, M>(0x811C9DC5u, x));
}

// The op on one lane's 4 consecutive elements of a row: x_1 = xr[0] .. xr[0]+3
// (xr[1..M-1] the row's other coordinates), `v` of them inside the simplex
// (v >= 1), at element offset `off` from `pin` / `pout`.  HASH with KF > 0:
// hpre[j] is the FNV-1a state after words x_1 + j, x_2 .. x_KF, common to
// the lane's rows.
template <int M, int OP, int KF = 0>
__device__ __forceinline__ void point_lane(int32_t n, const uint32_t *in, const uint32_t *pin, uint32_t *pout,
                                           uint32_t off, int32_t v, int32_t (&xr)[M],
                                           const uint32_t (&hpre)[4] = {0u, 0u, 0u, 0u})
{
    if (OP == OP_MAP) {
        asm volatile("" ::"v"(off), "v"(v));     // keep the mapping, drop nothing
    } else if (OP == OP_HITS) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < v) atomicAdd(pout + off + j, 1u);
    } else {
        uint32_t r[4];
        if (OP == OP_ACCUM) {
            if (v >= 4) {
                const uint4 q = *reinterpret_cast<const uint4 *>(pin + off);
                r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) r[j] = j < v ? pin[off + j] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] += 1u;
        } else if (OP == OP_EDM) {
            if constexpr (M == 2) {
                // element (x_1, x_2) holds d(p_i, p_j), i = x_1, j = n - x_2
                const float *pts = reinterpret_cast<const float *>(in);
                const int32_t jj = n - xr[1];
                const float qx = pts[3 * jj], qy = pts[3 * jj + 1], qz = pts[3 * jj + 2];
                auto dist = [&](float a, float b, float c) {
                    const float dx = a - qx, dy = b - qy, dz = c - qz;
                    return __float_as_uint(sqrtf(dx * dx + dy * dy + dz * dz));
                };
                const int32_t i0 = xr[0];
                if (v >= 4) {  // points i0 .. i0+3: 12 floats, 16-byte aligned (i0 % 4 == 0)
                    const float4 *q4 = reinterpret_cast<const float4 *>(pts + 3 * i0);
                    const float4 a = q4[0], b = q4[1], c = q4[2];
                    r[0] = dist(a.x, a.y, a.z);
                    r[1] = dist(a.w, b.x, b.y);
                    r[2] = dist(b.z, b.w, c.x);
                    r[3] = dist(c.y, c.z, c.w);
                } else {       // only the points inside: no read past point n
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float *p = pts + 3 * (i0 + (j < v ? j : 0));
                        r[j] = dist(p[0], p[1], p[2]);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) r[j] = 0u;
            }
        } else if constexpr (KF > 0) {  // OP_HASH from the lane's common leading words
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] = hash32_fmix(hash32_state<KF, M>(hpre[j], xr));
        } else {  // OP_HASH
            const int32_t x1 = xr[0];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xr[0] = x1 + j;
                r[j] = hash32_words<M>(xr);
            }
            xr[0] = x1;
        }
        if (v >= 4) {
            *reinterpret_cast<uint4 *>(pout + off) = make_uint4(r[0], r[1], r[2], r[3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < v) pout[off + j] = r[j];
        }
    }
}

// One tile (or one sub-block of a tile's rows) per NT-thread workgroup.  A
// lane handles 4 consecutive elements of a row along x_1 (one 16-byte
// access when all 4 lie in the simplex), G = rho/4 lanes cover a tile row,
// and the workgroup steps through the tile's rows NT/G at a time.  Row
// coordinates (x_2..x_m) are bit fields of the row index (rho is a power of
// two).  A lane whose 4 elements are all inside uses the vector access; a
// lane the hypotenuse cuts handles its elements one by one; lanes outside do
// nothing.  SUB workgroups share a tile, each taking a contiguous range of
// its rows.
template <int M, int RHO, int NT, int OP, bool BB, int SUB>
__global__ __launch_bounds__(NT) void k_point(const Plan P, const uint32_t *in, uint32_t *out)
{
    constexpr int G = RHO / 4;                   // lanes per tile row
    constexpr int LR = ilog2c(RHO);
    constexpr int ROWS = ipowc(RHO, M - 1);      // rows per tile
    constexpr int RPI = NT / G;                  // rows per workgroup iteration
    constexpr int RSUB = ROWS / SUB;             // rows per sub-block
    static_assert(RHO >= 4 && NT % G == 0 && ROWS % SUB == 0 && RSUB % RPI == 0, "bad tile shape");

    int32_t t[4] = {0, 0, 0, 0};
    uint32_t sub;
    if (BB) {
        const WgId g = wg_id(P);
        decode_bb(P, g.x, g.y, g.z / SUB, t);
        sub = g.z % SUB;
    } else {
        const WgId g = wg_id(P);
        if (!decode_h<M>(P, g.x / SUB, t)) return;
        sub = g.x % SUB;
    }
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
    const uint32_t *pin = in + base;
    uint32_t *pout = out + base;

    const int cx = threadIdx.x % G;
    const int32_t lx = 4 * cx;                       // tile-local x_1 of the lane's first element
#pragma unroll 4
    for (int it = 0; it < RSUB / RPI; ++it) {
        const uint32_t ri = sub * RSUB + it * RPI + threadIdx.x / G;   // tile-local row index
        int32_t rs = s0 + lx;                        // coordinate sum of the lane's first element
        uint32_t off = (uint32_t)lx;                 // tile-local element offset
        int32_t xr[M];
        xr[0] = x0[0] + lx;
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const int32_t l = (int32_t)((ri >> ((k - 1) * LR)) & (RHO - 1));
            xr[k] = x0[k] + l;
            rs += l;
            off += (uint32_t)l * (uint32_t)P.stride[k];
        }
        const int32_t v = n - rs + 1;                // elements of the lane inside the simplex
        if (v <= 0) continue;
        point_lane<M, OP>(n, in, pin, pout, off, v, xr);
    }
}

// Select the lane's value among U workgroup-uniform ones (u < U, unrolled:
// no runtime-indexed array).
template <int U, typename T>
__device__ __forceinline__ T pick_u(const T (&v)[U], int u)
{
    T r = v[0];
#pragma unroll
    for (int k = 1; k < U; ++k) r = (u == k) ? v[k] : r;
    return r;
}

// U tiles per NT-thread workgroup: map units U g .. U g + U - 1 (H: map
// indices; BB: the box tiles t_1 = U g_x .. U g_x + U - 1 of a row of the
// tile grid).  The map lays consecutive units x_1-adjacent wherever it can
// (the cube cells of a level run along x_1; a folded run is reversed), so
// the lanes of a wave stand side by side across the U tiles: a strip row
// is U tile rows of 4 rho bytes each, G lanes per tile, and a wave's store
// covers U times the contiguous bytes of one tile row (64 bytes instead of
// 32 at rho = 8, U = 2, m = 4).  The U decodes are
// workgroup-uniform scalar code, and each lane selects its own tile's
// origin once; units past the end of the grid, discarded units and tiles
// outside the simplex leave their lanes idle.  The strip rows a lane visits
// share their low row coordinates (the iteration advances the high ones), so
// the hash's leading words stay common to the lane's rows.
template <int M, int RHO, int NT, int OP, bool BB, int U>
__global__ __launch_bounds__(NT) void k_point_grp(const Plan P, const uint32_t *in, uint32_t *out)
{
    constexpr int G = RHO / 4;                   // lanes per tile row
    constexpr int SL = G * U;                    // lanes per strip row
    constexpr int LR = ilog2c(RHO);
    constexpr int ROWS = ipowc(RHO, M - 1);      // rows per tile
    constexpr int RPI = NT / SL;                 // strip rows per workgroup iteration
    static_assert(RHO >= 4 && U >= 2 && 64 % SL == 0 && NT % SL == 0 && ROWS % RPI == 0, "bad grouped shape");

    const int32_t n = P.n;
    int32_t tx[M][U];
    bool tv[U];
    const WgId g = wg_id(P);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int32_t t[4] = {0, 0, 0, 0};
        bool ok;
        if (BB) {
            const uint32_t gx = g.x * U + (uint32_t)u;
            ok = gx < (uint32_t)P.kbox;
            decode_bb(P, gx, g.y, g.z, t);
        } else {
            const uint32_t w = g.x * U + (uint32_t)u;
            ok = w < P.total && decode_h<M>(P, w, t);
        }
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            tx[k][u] = t[k] * RHO;
            s += t[k] * RHO;
        }
        tv[u] = ok && s <= n;
    }
    const int lu = (int)(threadIdx.x / G) % U;
    if (!pick_u<U>(tv, lu)) return;                  // no tile for this lane (no barriers below)
    int32_t x0[M];
    int32_t s0 = 0;
    int64_t base = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        x0[k] = pick_u<U>(tx[k], lu);
        s0 += x0[k];
        base += (int64_t)x0[k] * P.stride[k];
    }
    const uint32_t *pin = in + base;
    uint32_t *pout = out + base;

    const int32_t lx = 4 * (int)(threadIdx.x % G);  // tile-local x_1 of the lane's first element
    const uint32_t srow = threadIdx.x / SL;
    // Row coordinate k (k >= 1) is bit field [(k-1) LR, k LR) of the row
    // index srow + it RPI; the fields below log2(RPI) come from srow alone,
    // so coordinates x_1 .. x_KF are the same in every row the lane visits.
    constexpr int KF = 1 + ilog2c(RPI) / LR < M ? 1 + ilog2c(RPI) / LR : M - 1;
    uint32_t hpre[4] = {0u, 0u, 0u, 0u};
    if constexpr (OP == OP_HASH) {
        int32_t xf[M];
        xf[0] = x0[0] + lx;
#pragma unroll
        for (int k = 1; k < M; ++k) xf[k] = x0[k] + (int32_t)((srow >> ((k - 1) * LR)) & (RHO - 1));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hpre[j] = hash32_state<1, KF>((0x811C9DC5u ^ (uint32_t)(xf[0] + j)) * 0x01000193u, xf);
        }
    }
#pragma unroll
    for (int it = 0; it < ROWS / RPI; ++it) {
        const uint32_t ri = srow + (uint32_t)(it * RPI);   // tile-local row index
        int32_t rs = s0 + lx;
        uint32_t off = (uint32_t)lx;
        int32_t xr[M];
        xr[0] = x0[0] + lx;
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const int32_t l = (int32_t)((ri >> ((k - 1) * LR)) & (RHO - 1));
            xr[k] = x0[k] + l;
            rs += l;
            off += (uint32_t)l * (uint32_t)P.stride[k];
        }
        const int32_t v = n - rs + 1;
        if (v <= 0) continue;
        point_lane<M, OP, OP == OP_HASH ? KF : 0>(n, in, pin, pout, off, v, xr, hpre);
    }
}

}  // namespace smap
