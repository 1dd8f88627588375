// smap_ca3.hpp -- one step of the 3-D rule B6/S567 on Delta_n^3, uint8 cells.
//
// The CA test of Section 5.1 on the 3-simplex: 26-neighbourhood, cells
// outside the simplex dead (the "fixed dead cells" boundary), birth on 6
// live neighbours, survival on 5, 6 or 7.
//
// Work split.  The map (H or BB) gives a rho^3 tile; the tile is split into
// sub-blocks of rho (x) x RY (y) x RZ (z) cells, one workgroup each.  The
// launch orders the sub-block index slowest, so workgroups that run together
// cover neighbouring tiles of the same sub-block position.  The workgroup
// walks its RZ planes along z.  Each plane of its slab, with one halo row on
// each side in y and four halo bytes on each side in x, is staged in LDS:
// the (RY+2) rows of x0-4 .. x0+rho+4 are cut into 16-byte chunks that the
// lanes load from global memory (unaligned 16-byte accesses), clear outside
// the simplex, and write to LDS.  Every staged byte is read from global
// memory once per workgroup, and the zeroed cells outside the simplex make
// the neighbour sums need no boundary test.  Two LDS buffers alternate, with
// one barrier per plane; the chunk loads of the next two planes are in
// flight while a plane is summed.
//
// A lane owns 16 consecutive cells of RL consecutive rows (x .. x+15 at
// y .. y+RL-1); rho/16 lanes cover RL tile rows.  From LDS it reads, for each
// of its RL+2 rows, 24 bytes: the dword left of its cells, the 16 cells and
// the dword right of them, and forms the in-plane 3x3 box sums S(z) of its
// RL rows (<= 9 per byte).  The 3x3x3 sum including the centre is
// S(z-1)+S(z)+S(z+1) (<= 27); the sums of the two previous planes stay in
// registers as the walk proceeds.
//
// Stores go straight from registers: a 16-byte store when the lane's cells
// are all inside, the cells inside one by one on the lane the hypotenuse
// cuts, nothing outside.  The SAFE instantiation (n < 15) loads byte by byte
// near the end of the buffer.
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

// Shape constants of a CA3 tile walk.
template <int RHO, int RY, int RZ, int RL>
struct Ca3Walk {
    static constexpr int G = RHO / 16;                 // lanes per tile row
    static constexpr int NT = G * (RY / RL);           // threads
    static constexpr int SUBY = RHO / RY, SUBZ = RHO / RZ, SUB = SUBY * SUBZ;
    static_assert(G >= 2 && 64 % G == 0 && NT % 64 == 0 && RY % RL == 0 && RHO % RY == 0 &&
                  RHO % RZ == 0, "bad CA3 tile shape");
};

// One B6/S567 step of sub-block `sub` of the rho^3 tile t (workgroup body;
// every thread of the workgroup must call it: it has barriers).
template <int RHO, int RY, int RZ, int RL, bool SAFE, int PD = 2>
__device__ __forceinline__ void ca3_tile(const Plan &P, const uint8_t *__restrict__ in,
                                         uint8_t *__restrict__ out, const int32_t *t, uint32_t sub)
{
    static_assert(PD >= 2 && PD <= 4, "prefetch depth");
    using Sh = Ca3Walk<RHO, RY, RZ, RL>;
    constexpr int G = Sh::G, NT = Sh::NT, SUBY = Sh::SUBY;
    constexpr int C = (RHO + 8 + 15) / 16;      // 16-byte chunks per staged row (x0-4 .. x0+rho+4)
    constexpr int PITCH = 16 * C;               // LDS bytes per staged row
    constexpr int ROWS = RY + 2;                // staged rows y0-1 .. y0+RY
    constexpr int NCH = ROWS * C;               // chunks per staged plane
    constexpr int KQ = (NCH + NT - 1) / NT;     // chunks per lane per plane
    __shared__ __align__(16) uint8_t lds[2][ROWS * PITCH];

    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO;
    const int32_t y0 = t[1] * RHO + (int32_t)(sub % SUBY) * RY;
    const int32_t z0 = t[2] * RHO + (int32_t)(sub / SUBY) * RZ;
    if (x0 + y0 + z0 > n) return;                 // uniform: no cell in this sub-block
    // output planes with a simplex cell: z0 .. z0 + nz - 1 (workgroup-uniform)
    const int32_t nz = min(RZ, n - x0 - y0 - z0 + 1);
    // last staged plane that an output plane reads: z0 + nz (the halo above),
    // or n; planes beyond it are never loaded
    const int32_t zhi = min(n, z0 + nz);
    const int64_t p1 = P.stride[1], p2 = P.stride[2];
    const int64_t total = p2 * p1;
    const int tid = threadIdx.x;

    // Chunk k of this lane: staged row r = q / C, chunk column c = q % C,
    // covering y = y0-1+r, x = x0-4+16c .. +15 (q = tid + k NT < NCH).
    // Returns the row y, the first x and the in-plane offset of the load
    // (x clamped to 0 for the left halo chunk of a tile at x0 = 0).
    auto chunk_geom = [&](int k, int32_t &y, int32_t &xs, uint32_t &off) {
        const int q = tid + k * NT;
        const int r = q / C, c = q % C;
        y = y0 - 1 + r;
        xs = x0 - 4 + 16 * c;
        off = (uint32_t)max(y, 0) * (uint32_t)p1 + (uint32_t)max(xs, 0);
    };
    // Raw loads of the lane's chunks of plane z (no masking: the loads of a
    // plane issue back to back).  Outside the byte-safe instantiation every
    // lane issues all KQ loads, reading the buffer's first 16 bytes for a
    // chunk with no simplex cell (or a plane outside 0..n); commit_plane
    // clears such chunks.  Unconditional loads keep the number of loads
    // issued after a register set known, so the wait before its use is a
    // partial one and the loads of the next planes stay in flight.
    auto load_plane = [&](int32_t z, uint4 (&R)[KQ]) {
        const bool zin = (uint32_t)z <= (uint32_t)zhi;  // uniform
        if constexpr (SAFE) {
#pragma unroll
            for (int k = 0; k < KQ; ++k) R[k] = make_uint4(0u, 0u, 0u, 0u);
            if (!zin) return;
#pragma unroll
            for (int k = 0; k < KQ; ++k) {
                if (NCH % NT != 0 && tid + k * NT >= NCH) continue;
                int32_t y, xs;
                uint32_t off;
                chunk_geom(k, y, xs, off);
                const int32_t xl = max(xs, 0);
                if (y < 0 || n - z - y - xl < 0) continue;
                const int64_t rb = (int64_t)z * p2 + (int64_t)y * p1;
                R[k].x = ld_masked(in + rb, xl, y + z, n, total - rb);
                R[k].y = ld_masked(in + rb, xl + 4, y + z, n, total - rb);
                R[k].z = ld_masked(in + rb, xl + 8, y + z, n, total - rb);
                R[k].w = ld_masked(in + rb, xl + 12, y + z, n, total - rb);
            }
        } else {
            const uint8_t *pl = in + (int64_t)(zin ? z : 0) * p2;   // uniform
#pragma unroll
            for (int k = 0; k < KQ; ++k) {
                int32_t y, xs;
                uint32_t off;
                chunk_geom(k, y, xs, off);
                const bool has = zin && (NCH % NT == 0 || tid + k * NT < NCH) && y >= 0 &&
                                 n - z - y - max(xs, 0) >= 0;
                uint64_t a = has ? (uint64_t)(pl - in) + off : 0u;
                // The offset is opaque to the compiler: a plane with no cell
                // in this sub-block (a uniform offset 0) would otherwise
                // become a scalar load on a branch of its own, and a path
                // that issues no vector load turns every later wait for a
                // load into a full drain of the loads in flight.
                asm("" : "+v"(a));
                R[k] = *reinterpret_cast<const uint4 *>(in + a);
            }
        }
    };
    // Clear the bytes outside the simplex and write the chunks of plane z to
    // LDS buffer b.  Every chunk slot is written (zeros where nothing was
    // loaded).
    auto commit_plane = [&](int32_t z, const uint4 (&R)[KQ], int b) {
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            if (NCH % NT != 0 && tid + k * NT >= NCH) continue;
            int32_t y, xs;
            uint32_t off;
            chunk_geom(k, y, xs, off);
            uint32_t w[4] = {R[k].x, R[k].y, R[k].z, R[k].w};
            if (xs < 0) {                         // loaded from x = 0: shift into place
                w[3] = w[2];
                w[2] = w[1];
                w[1] = w[0];
                w[0] = 0u;
            }
            // cells x_s .. x_s + v - 1 of the chunk are in the simplex
            const int32_t v = ((uint32_t)z > (uint32_t)zhi || y < 0) ? 0 : n - z - y - xs + 1;
            if (v < 16) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int32_t keep = v - 4 * i;
                    w[i] = keep >= 4 ? w[i] : (keep <= 0 ? 0u : w[i] & ((1u << (8 * keep)) - 1u));
                }
            }
            const int q = tid + k * NT;
            *reinterpret_cast<uint4 *>(&lds[b][(q / C) * PITCH + (q % C) * 16]) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    };

    const int cx = tid % G, rp = tid / G;
    const int32_t x = x0 + 16 * cx;
    const int32_t ylane = y0 + rp * RL;           // first output row of the lane
    // In-plane 3x3 sums of the lane's RL rows from LDS buffer b, and the
    // centre cells of those rows.
    auto plane_sums = [&](int b, uint32_t (&S)[RL][4], uint32_t (&ctr)[RL][4]) {
        uint32_t h[RL + 2][4];
#pragma unroll
        for (int jj = 0; jj < RL + 2; ++jj) {
            const uint8_t *src = &lds[b][(rp * RL + jj) * PITCH + 16 * cx];
            const uint4 a = *reinterpret_cast<const uint4 *>(src);        // left dword, cells 0..11
            const uint2 e = *reinterpret_cast<const uint2 *>(src + 16);   // cells 12..15, right dword
            const uint32_t c[4] = {a.y, a.z, a.w, e.x};
            hsum16(c, a.x, e.y, h[jj]);
            if (jj >= 1 && jj <= RL) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ctr[jj - 1][i] = c[i];
            }
        }
#pragma unroll
        for (int j = 0; j < RL; ++j) {
#pragma unroll
            for (int i = 0; i < 4; ++i) S[j][i] = h[j][i] + h[j + 1][i] + h[j + 2][i];
        }
    };

    // PD register sets of chunk loads rotate (the plane loop is unrolled by
    // PD), so a set is consumed PD planes after its loads were issued with no
    // register copy in between: a copy would wait for the loads.
    uint4 RS[PD][KQ];
    load_plane(z0 - 1, RS[0]);
    commit_plane(z0 - 1, RS[0], 0);
#pragma unroll
    for (int u = 0; u < PD; ++u) load_plane(z0 + u, RS[u]);
    lds_barrier();

    uint32_t sp[RL][4] = {}, sc[RL][4] = {}, cp[RL][4] = {};
    // Staged planes z0-1 .. z0+nz; the walk runs a multiple of PD steps so
    // that every part of the unrolled loop always runs (a step beyond the
    // last plane stages zeros and stores nothing), and every step issues
    // its loads: the wait before a register set's use then only covers that
    // set, not the loads issued after it.
    const int32_t steps = (nz + 2 + PD - 1) / PD * PD;
    // Step i: plane z0-1+i is staged in lds[i & 1] and RX holds plane z0+i.
    auto step = [&](int32_t i, uint4 (&RX)[KQ]) {
        uint32_t sn[RL][4], cn[RL][4];
        plane_sums(i & 1, sn, cn);
        if (i >= 2 && i < nz + 2) {               // output plane z0 + i - 2
            const int32_t z = z0 + i - 2;
#pragma unroll
            for (int j = 0; j < RL; ++j) {
                uint32_t res[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) res[k] = rule_b6s567(sp[j][k] + sc[j][k] + sn[j][k], cp[j][k]);
                const int32_t yj = ylane + j;
                const int32_t v = n - z - yj - x + 1;
                if (v > 0) {
                    uint8_t *row = out + (int64_t)z * p2 + (int64_t)yj * p1;
                    if (v >= 16) {
                        *reinterpret_cast<uint4 *>(row + x) = make_uint4(res[0], res[1], res[2], res[3]);
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) st_masked(row, x + 4 * k, yj + z, n, res[k]);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RL; ++j) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sp[j][k] = sc[j][k];
                sc[j][k] = sn[j][k];
                cp[j][k] = cn[j][k];
            }
        }
        commit_plane(z0 + i, RX, (i + 1) & 1);   // staged for step i + 1
        load_plane(z0 + i + PD, RX);              // consumed at step i + PD
        lds_barrier();
    };
    for (int32_t i = 0; i < steps; i += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) step(i + u, RS[u]);
    }
}

// The CA3 kernel.  BB: grid (kbox, kbox, kbox * SUB).  H: grid (map grid,
// SUB); x-adjacent tiles of one sub-block position run together.
template <int RHO, int RY, int RZ, int RL, bool BB, bool SAFE>
__global__ __launch_bounds__((RHO / 16) * (RY / RL)) void k_ca3(const Plan P, const uint8_t *__restrict__ in,
                                                                       uint8_t *__restrict__ out)
{
    constexpr int SUB = Ca3Walk<RHO, RY, RZ, RL>::SUB;
    int32_t t[4] = {0, 0, 0, 0};
    uint32_t sub;
    const WgId g = wg_id(P);
    if (BB) {
        decode_bb(P, g.x, g.y, g.z / SUB, t);
        sub = g.z % SUB;
    } else {
        if (!decode_h<3>(P, g.x, t)) return;
        sub = g.y;
    }
    ca3_tile<RHO, RY, RZ, RL, SAFE>(P, in, out, t, sub);
}

}  // namespace smap
