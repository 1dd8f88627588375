// smap_ca3.hpp -- one step of the 3-D rule B6/S567 on Delta_n^3, uint8 cells.
//
// The CA test of Section 5.1 on the 3-simplex: 26-neighbourhood, cells
// outside the simplex dead (the "fixed dead cells" boundary), birth on 6
// live neighbours, survival on 5, 6 or 7.
//
// Work split.  The map (H or BB) gives a rho^3 tile; the tile is split into
// sub-blocks of rho (x) x RY (y) x RZ (z) cells, one workgroup each.  The
// launch orders the sub-block index slowest, so workgroups that run together
// cover neighbouring tiles of the same sub-block position.  A lane owns 16
// consecutive cells of RL consecutive rows (x .. x+15 at y .. y+RL-1, fixed
// z); a group of rho/16 lanes covers RL tile rows.  The workgroup walks its
// RZ planes along z.  For each input plane a lane reads the rows y-1 ..
// y+RL straight from global memory (16-byte accesses; the outer two rows
// are other lanes' rows, so those re-reads are served by the caches), takes
// the left/right neighbour bytes from the adjacent lanes by DPP (halo bytes
// by one extra load at the row-group edges), and forms the in-plane 3x3 box
// sum S(z) of each of its rows (<= 9 per byte).  The 3x3x3 sum including
// the centre is S(z-1)+S(z)+S(z+1) (<= 27); the sums of the two previous
// planes stay in registers as the walk proceeds.

// Boundary handling is per lane, as in the 2-D kernel: inside lanes use
// plain 16-byte accesses, the lane the hypotenuse cuts masks its bytes,
// lanes outside touch nothing; the SAFE instantiation (n < 15) reads byte by
// byte near the end of the buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_decode.hpp"

namespace smap {

// B6/S567 on four byte cells: t = 3x3x3 sum including the centre (<= 27),
// c = centre (0/1).  next = 1 iff t >= 6 and t - 6 <= 2c.  With
// d = t + 0x7A per byte, bit 7 of d is (t >= 6); e = d - (2c + 1) has bit 7
// clear iff t - 6 <= 2c (no byte borrows or carries: 0x77 <= e, d <= 0x95).
__device__ __forceinline__ uint32_t rule_b6s567(uint32_t t, uint32_t c)
{
    const uint32_t d = t + 0x7A7A7A7Au;
    const uint32_t e = d - ((c << 1) | 0x01010101u);
    return ((d & ~e) >> 7) & 0x01010101u;
}

template <int RHO, int RY, int RZ, int RL, bool BB, bool SAFE>
__global__ __launch_bounds__((RHO / 16) * (RY / RL)) void k_ca3(const Plan P, const uint8_t *__restrict__ in,
                                                                uint8_t *__restrict__ out)
{
    constexpr int G = RHO / 16;            // lanes per tile row
    constexpr int NR = RL + 2;             // rows read per plane by a lane
    constexpr int SUBY = RHO / RY, SUBZ = RHO / RZ, SUB = SUBY * SUBZ;
    static_assert(G >= 2 && 64 % G == 0 && (G * (RY / RL)) % 64 == 0 && RY % RL == 0 &&
                  RHO % RY == 0 && RHO % RZ == 0, "bad CA3 tile shape");

    int32_t t[4] = {0, 0, 0, 0};
    uint32_t sub;
    if (BB) {
        const WgId g = wg_id(P);
        decode_bb(P, g.x, g.y, g.z / SUB, t);
        sub = g.z % SUB;
    } else {  // grid (map grid, SUB): x-adjacent tiles of one sub-block run together
        const WgId g = wg_id(P);
#ifdef SMAP_CA3_TILE_MAJOR
        if (!decode_h<3>(P, g.x / SUB, t)) return;
        sub = g.x % SUB;
#else
        if (!decode_h<3>(P, g.x, t)) return;
        sub = g.y;
#endif
    }
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO;
    const int32_t y0 = t[1] * RHO + (int32_t)(sub % SUBY) * RY;
    const int32_t z0 = t[2] * RHO + (int32_t)(sub / SUBY) * RZ;
    if (x0 + y0 + z0 > n) return;                 // uniform: no cell in this sub-block
    // output planes with a simplex cell: z0 .. z0 + nz - 1 (workgroup-uniform)
    const int32_t nz = min(RZ, n - x0 - y0 - z0 + 1);

    const int tid = threadIdx.x;
    const int cx = tid % G, rp = tid / G;
    const int32_t x = x0 + 16 * cx;
    const int32_t y = y0 + rp * RL;               // first output row of the lane
    const int32_t xe = (cx == 0) ? x0 - 4 : x0 + RHO;
    const bool is_edge = (cx == 0) || (cx == G - 1);
    const int64_t p1 = P.stride[1], p2 = P.stride[2];
    const int64_t total = p2 * p1;
    // per-lane 32-bit offsets, inside a plane, of the rows y-1 .. y+RL read
    // for every plane (rows never read are clamped to 0)
    uint32_t off[NR], offe[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int32_t yy = y - 1 + k;
        off[k] = yy >= 0 ? (uint32_t)yy * (uint32_t)p1 + (uint32_t)x : 0u;
        offe[k] = (yy >= 0 && xe >= 0) ? (uint32_t)yy * (uint32_t)p1 + (uint32_t)xe : 0u;
    }

    // Raw loads of the rows of plane z the lane needs.
    auto load_plane = [&](int32_t z, uint32_t (&c)[NR][4], uint32_t (&e)[NR]) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            c[k][0] = c[k][1] = c[k][2] = c[k][3] = 0u;
            e[k] = 0u;
        }
        if ((uint32_t)z > (uint32_t)n) return;      // z < 0 or z > n (uniform)
        const uint8_t *pl = in + (int64_t)z * p2;    // wave-uniform plane pointer
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int32_t yy = y - 1 + k;
            if (yy < 0 || yy > n) continue;
            const int32_t lim = n - z - yy;          // largest x of the row in the simplex
            if constexpr (SAFE) {
                const int64_t rb = (int64_t)z * p2 + (int64_t)yy * p1;
#pragma unroll
                for (int i = 0; i < 4; ++i) c[k][i] = ld_masked(in + rb, x + 4 * i, yy + z, n, total - rb);
                if (is_edge) e[k] = ld_masked(in + rb, xe, yy + z, n, total - rb);
            } else {
                if (x <= lim) {
                    const uint4 q = *reinterpret_cast<const uint4 *>(pl + off[k]);
                    c[k][0] = q.x; c[k][1] = q.y; c[k][2] = q.z; c[k][3] = q.w;
                }
                if (is_edge && xe >= 0 && xe <= lim) e[k] = ld_u32(pl + offe[k]);
            }
        }
    };
    // Zero the cells outside the simplex, then form the in-plane 3x3 sums of
    // the lane's RL rows (and their centre rows).
    auto plane_sums = [&](int32_t z, uint32_t (&c)[NR][4], uint32_t (&e)[NR], uint32_t (&S)[RL][4],
                          uint32_t (&ctr)[RL][4]) {
        uint32_t h[NR][4];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if constexpr (!SAFE) {
                const int32_t v = n - z - (y - 1 + k) - x + 1;
                if (v < 16) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int32_t keep = v - 4 * i;
                        c[k][i] = keep >= 4 ? c[k][i] : (keep <= 0 ? 0u : c[k][i] & ((1u << (8 * keep)) - 1u));
                    }
                }
                const int32_t ve = n - z - (y - 1 + k) - xe + 1;
                if (ve < 4) e[k] = ve <= 0 ? 0u : e[k] & ((1u << (8 * ve)) - 1u);
            }
            hsum16(c[k], lane_prev<G>(c[k], e[k], cx), lane_next<G>(c[k], e[k], cx), h[k]);
        }
#pragma unroll
        for (int j = 0; j < RL; ++j) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                S[j][i] = h[j][i] + h[j + 1][i] + h[j + 2][i];
                ctr[j][i] = c[j + 1][i];
            }
        }
    };

    // planes z0-1 and z0: the first two in-plane sums
    uint32_t sp[RL][4], sc[RL][4], cc[RL][4];
    {
        uint32_t ca[NR][4], ea[NR], junk[RL][4];
        load_plane(z0 - 1, ca, ea);
        plane_sums(z0 - 1, ca, ea, sp, junk);
        load_plane(z0, ca, ea);
        plane_sums(z0, ca, ea, sc, cc);
    }
    for (int32_t p = 0; p < nz; ++p) {
        const int32_t z = z0 + p;                    // output plane
        uint32_t cn[NR][4], en[NR], sn[RL][4], cnext[RL][4];
        load_plane(z + 1, cn, en);
        plane_sums(z + 1, cn, en, sn, cnext);
#pragma unroll
        for (int j = 0; j < RL; ++j) {
            uint32_t res[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) res[i] = rule_b6s567(sp[j][i] + sc[j][i] + sn[j][i], cc[j][i]);
            // store the lane's cells of row (y + j, z) that lie in the simplex
            const int32_t yj = y + j;
            const int32_t v = n - z - yj - x + 1;
            if (yj <= n && v > 0) {
                uint8_t *row = out + (int64_t)z * p2 + (int64_t)yj * p1;
                if (v >= 16) {
                    *reinterpret_cast<uint4 *>(row + x) = make_uint4(res[0], res[1], res[2], res[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) st_masked(row, x + 4 * i, yj + z, n, res[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sp[j][i] = sc[j][i];
                sc[j][i] = sn[j][i];
                cc[j][i] = cnext[j][i];
            }
        }
    }
}

}  // namespace smap
