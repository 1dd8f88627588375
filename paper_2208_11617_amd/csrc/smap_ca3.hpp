// smap_ca3.hpp -- one step of the 3-D rule B6/S567 on Delta_n^3, uint8 cells.
//
// The CA test of Section 5.1 on the 3-simplex: 26-neighbourhood, cells
// outside the simplex dead (the "fixed dead cells" boundary), birth on 6
// live neighbours, survival on 5, 6 or 7.
//
// Work split.  A workgroup of 256 threads owns a 32^3 tile (from H or BB)
// and walks it along x_3 (z).  For each plane z it stages the 34 x 34 halo
// plane (x and y extended by one cell each side) in LDS -- as 34 rows of 10
// dwords, the first and last dword of a row carrying the halo bytes -- with
// two LDS buffers so one barrier per plane suffices and the global loads of
// plane z+1 are in flight while plane z is summed.  Thread (cx, ry) owns the
// 4 cells at x = x0 + 4 cx, y = y0 + ry and reads its 3 x 3 x (6 bytes)
// neighbourhood from LDS, forming the in-plane 3x3 box sum S(z) per byte
// (<= 9).  The 3x3x3 sum including the centre is S(z-1) + S(z) + S(z+1)
// (<= 27), kept in registers as the walk proceeds; next = (t == 6) |
// (alive & (t == 7 | t == 8)).
//
// Boundary handling as in the 2-D kernel: planes whose whole halo plane lies
// inside the simplex load plain dwords; others zero the cells outside it;
// stores write only cells inside (byte stores for a partial last dword).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_decode.hpp"

namespace smap {

__device__ __forceinline__ uint32_t rule_b6s567(uint32_t t, uint32_t c)
{
    const uint32_t ne6 = (t ^ 0x06060606u) + 0x7F7F7F7Fu;
    const uint32_t ne7 = (t ^ 0x07070707u) + 0x7F7F7F7Fu;
    const uint32_t ne8 = (t ^ 0x08080808u) + 0x7F7F7F7Fu;
    return ((~ne6 | ((~ne7 | ~ne8) & (c << 7))) >> 7) & 0x01010101u;
}

template <bool BB>
__global__ __launch_bounds__(256) void k_ca3_32(const Plan P, const uint8_t *__restrict__ in,
                                                uint8_t *__restrict__ out)
{
    constexpr int RHO = 32;
    constexpr int DW = RHO / 4 + 2;   // dwords per staged row (with both halo dwords)
    constexpr int HR = RHO + 2;       // staged rows
    constexpr int NQ = HR * DW;       // dwords per staged plane (340)
    __shared__ uint32_t lds[2][NQ];

    int32_t t[4] = {0, 0, 0, 0};
    if (!wg_tile<3, BB>(P, t)) return;
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO, y0 = t[1] * RHO, z0 = t[2] * RHO;
    if (x0 + y0 + z0 > n) return;                 // uniform: before any barrier

    const int tid = threadIdx.x;
    const int cx = tid & 7, ry = tid >> 3;
    const int64_t p1 = P.stride[1], p2 = P.stride[2];
    const int64_t total = p2 * p1;

    // staged dwords of this thread: q0 = tid, q1 = tid + 256 (if < NQ)
    const int q1 = tid + 256;
    const bool has_q1 = q1 < NQ;
    const int hr0 = tid / DW, hc0 = tid % DW;
    const int hr1 = q1 / DW, hc1 = q1 % DW;
    const int32_t gx0 = x0 - 4 + 4 * hc0, gy0 = y0 - 1 + hr0;
    const int32_t gx1 = x0 - 4 + 4 * hc1, gy1 = y0 - 1 + hr1;

    const int32_t zlast = min(z0 + RHO - 1, n - x0 - y0);  // last plane with simplex cells
    const int nplanes = zlast - z0 + 3;                      // z0-1 .. zlast+1

    auto load_plane = [&](int32_t z, uint32_t &v0, uint32_t &v1) {
        const bool fast = x0 >= 4 && y0 >= 1 && z >= 0 && (x0 + RHO) + (y0 + RHO) + z <= n;
        const int64_t zb = (int64_t)z * p2;
        if (fast) {
            v0 = ld_u32(in + zb + (int64_t)gy0 * p1 + gx0);
            v1 = has_q1 ? ld_u32(in + zb + (int64_t)gy1 * p1 + gx1) : 0u;
        } else if (z < 0 || z > n) {
            v0 = 0u;
            v1 = 0u;
        } else {
            v0 = 0u;
            v1 = 0u;
            if (gy0 >= 0 && gy0 <= n) {
                const int64_t rb = zb + (int64_t)gy0 * p1;
                v0 = ld_masked(in + rb, gx0, gy0 + z, n, total - rb);
            }
            if (has_q1 && gy1 >= 0 && gy1 <= n) {
                const int64_t rb = zb + (int64_t)gy1 * p1;
                v1 = ld_masked(in + rb, gx1, gy1 + z, n, total - rb);
            }
        }
    };

    uint32_t v0, v1;
    load_plane(z0 - 1, v0, v1);
    uint32_t s_prev = 0u, s_cur = 0u, c_cur = 0u;
    const int32_t x = x0 + 4 * cx, y = y0 + ry;
    const int64_t lane_off = (int64_t)y * p1 + x;

    for (int p = 0; p < nplanes; ++p) {
        const int32_t z = z0 - 1 + p;
        uint32_t *buf = lds[p & 1];
        buf[tid] = v0;
        if (has_q1) buf[q1] = v1;
        __syncthreads();
        if (p + 1 < nplanes) load_plane(z + 1, v0, v1);

        uint32_t s = 0u, c = 0u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t *row = buf + (ry + k) * DW + cx;
            const uint32_t l = row[0], m = row[1], r = row[2];
            s += __builtin_amdgcn_alignbyte(m, l, 3) + m + __builtin_amdgcn_alignbyte(r, m, 1);
            if (k == 1) c = m;
        }
        if (p >= 2) {  // output plane z - 1
            const int32_t zo = z - 1;
            const uint32_t res = rule_b6s567(s_prev + s_cur + s, c_cur);
            uint8_t *dst = out + (int64_t)zo * p2 + lane_off;
            const int32_t v = n - x - y - zo + 1;
            if (v >= 4) {
                st_u32(dst, res);
            } else if (v > 0) {
                for (int k = 0; k < v; ++k) dst[k] = (uint8_t)(res >> (8 * k));
            }
        }
        s_prev = s_cur;
        s_cur = s;
        c_cur = c;
    }
}

}  // namespace smap
