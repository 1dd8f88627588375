// smap_ca3k.hpp -- several B6/S567 generations per pass over HBM (3-D).
//
// The paper's automaton test runs a fixed number of steps (Section 5.1);
// this is that loop on the 3-simplex, blocked in time.  One launch advances
// every cell of Delta_n^3 by `gens` <= KH generations: a workgroup loads its
// rho^3 tile plus a halo of KH cells on every side into LDS (cells outside
// the simplex, or outside the box, dead), steps the region `gens` times in
// LDS and writes the tile.  After generation g the cells within g of the
// region's faces are stale, so with gens <= KH the tile itself is exact.
// HBM bytes per generation: ((rho + 2 KH)^3 / rho^3 + 1) / gens per cell
// instead of 2.
//
// In LDS a cell is one bit: ONE buffer of W = rho + 2 KH planes x W rows x
// W/32 dwords (110,592 bytes for rho = 64, KH = 16); bit b of dword c of row
// y of plane z is the cell (x0 - KH + 32c + b, y0 - KH + y, z0 - KH + z).
// The count is bit-sliced, 32 cells per operation: a row's horizontal
// 3-sum is a full adder over the row and its copies shifted by one cell
// (2 bits per cell), the in-plane 3x3 sum adds three of those (4 bits, at
// most 9), and the 3x3x3 sum including the centre adds three in-plane sums
// (5 bits, at most 27).  A generation updates the region in place: a thread
// owns one dword of one row and walks the planes along z with the in-plane
// sums of the two previous planes in registers; the new plane z is written
// one step later, once every thread has read the old plane z, so threads
// up to one step apart never touch a plane another reads or writes (one
// barrier per two planes).  Three parts of the workgroup walk three ranges
// of the planes at once.  Generation g updates planes and rows g .. W-1-g
// only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_ca2k.hpp"
#include "smap_decode.hpp"

namespace smap {

template <int RHO, int KH>
struct Ca3kShape {
    static constexpr int W = RHO + 2 * KH;        // cells per staged row; rows; planes
    static constexpr int DW = W / 32;              // dwords (32 cells) per staged row
    static constexpr int NCOL = DW * (W - 2);      // thread columns: a dword of rows 1 .. W-2
    static constexpr int NP = 3;                   // parts of the plane walk, walked at once
    static constexpr int PART = ((NCOL + 63) / 64) * 64;   // threads per part
    static constexpr int NT = NP * PART;
    static_assert(W % 32 == 0 && KH % 16 == 0 && RHO % 32 == 0 && NT <= 1024, "bad CA3K shape");
};

// Simplex cells of the dword (x .. x+3, y, z): bytes kept.
__device__ __forceinline__ uint32_t ca3k_keep_mask(int32_t x, int32_t y, int32_t z, int32_t n)
{
    if (x < 0 || y < 0 || z < 0) return 0u;
    const int32_t keep = n - z - y - x + 1;
    return keep >= 4 ? 0xFFFFFFFFu : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
}

// Sum of three 2-bit bit-sliced numbers (a1 a0) + (b1 b0) + (c1 c0): 4 bits.
__device__ __forceinline__ void add3_2(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1, uint32_t c0, uint32_t c1,
                                       uint32_t (&q)[4])
{
    const uint32_t t0 = a0 ^ b0, k0 = a0 & b0;
    const uint32_t x1 = a1 ^ b1;
    const uint32_t t1 = x1 ^ k0, k1 = (a1 & b1) | (k0 & x1);
    q[0] = t0 ^ c0;
    const uint32_t m0 = t0 & c0;
    const uint32_t y1 = t1 ^ c1;
    q[1] = y1 ^ m0;
    const uint32_t m1 = (t1 & c1) | (m0 & y1);
    q[2] = k1 ^ m1;
    q[3] = k1 & m1;
}

template <int RHO, int KH, bool SAFE>
__device__ __forceinline__ void ca3k_tile(const Plan &P, const uint8_t *__restrict__ in,
                                          uint8_t *__restrict__ out, const int32_t *t, int gens)
{
    using Sh = Ca3kShape<RHO, KH>;
    constexpr int W = Sh::W, DW = Sh::DW, NT = Sh::NT;
    __shared__ uint32_t buf[W][W][DW];
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO, y0 = t[1] * RHO, z0 = t[2] * RHO;
    if (x0 + y0 + z0 > n) return;                // uniform: BB tile outside the simplex
    const int64_t p1 = P.stride[1], p2 = P.stride[2];
    const int64_t total = p2 * p1;
    const int tid = threadIdx.x;
    const int32_t xs = x0 - KH, ys = y0 - KH, zs = z0 - KH;   // cell of bit 0, dword 0, row 0, plane 0

    // 1. Stage the region.  A dword is two 16-byte chunks, each loaded from
    //    its first cell (x >= 0 for every chunk with a simplex cell, KH being
    //    a multiple of 16), cleared outside the simplex and packed to bits.
    //    From n = 15 on a 16-byte access from a simplex cell stays inside the
    //    buffer, so LB dwords' loads are issued unconditionally (the buffer's
    //    first 16 bytes for a chunk without a simplex cell) before any is
    //    used; below, bytes go through the masked load.
    constexpr int NL = W * W * DW, LB = 4;
    uint32_t *flat = &buf[0][0][0];
    for (int q0 = tid; q0 < NL; q0 += NT * LB) {
        uint4 v[LB][2];
        int32_t cx[LB], cy[LB], cz[LB];
#pragma unroll
        for (int k = 0; k < LB; ++k) {
            const int q = min(q0 + k * NT, NL - 1);
            const int c = q % DW, y = (q / DW) % W, z = q / (DW * W);
            cx[k] = xs + 32 * c;
            cy[k] = ys + y;
            cz[k] = zs + z;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t x = cx[k] + 16 * h;
                const bool has = cy[k] >= 0 && cz[k] >= 0 && x >= 0 && x <= n - cy[k] - cz[k];
                if constexpr (SAFE) {
                    v[k][h] = make_uint4(0u, 0u, 0u, 0u);
                    if (has) {
                        const int64_t rb = (int64_t)cz[k] * p2 + (int64_t)cy[k] * p1;
                        const int32_t r = cy[k] + cz[k];
                        v[k][h].x = ld_masked(in + rb, x, r, n, total - rb);
                        v[k][h].y = ld_masked(in + rb, x + 4, r, n, total - rb);
                        v[k][h].z = ld_masked(in + rb, x + 8, r, n, total - rb);
                        v[k][h].w = ld_masked(in + rb, x + 12, r, n, total - rb);
                    }
                } else {
                    const uint8_t *a = has ? in + ((int64_t)cz[k] * p2 + (int64_t)cy[k] * p1 + x) : in;
                    v[k][h] = *reinterpret_cast<const uint4 *>(a);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < LB; ++k) {
            uint32_t word = 0u;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t x = cx[k] + 16 * h;
                const uint32_t w[4] = {v[k][h].x, v[k][h].y, v[k][h].z, v[k][h].w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    word |= pack4(w[i] & ca3k_keep_mask(x + 4 * i, cy[k], cz[k], n)) << (16 * h + 4 * i);
            }
            if (q0 + k * NT < NL) flat[q0 + k * NT] = word;
        }
    }
    __syncthreads();

    // 2. Generations.  Thread column: dword c of row y.  The planes of a
    //    generation are cut into NP consecutive ranges, walked by NP parts of
    //    the workgroup at once.  A part keeps its first new plane in a
    //    register until the generation ends (the part below reads that
    //    plane's old cells at its last step), and every part writes its last
    //    new plane only then (the part above read it at its first step).
    const int part = tid / Sh::PART, lt = tid % Sh::PART;
    const bool worker = lt < Sh::NCOL;
    const int c = lt % DW;
    const int y = 1 + lt / DW;
    const int32_t gx = xs + 32 * c;
    const bool interior = xs >= 0 && ys >= 0 && zs >= 0 && xs + ys + zs + 3 * (W - 1) <= n;   // uniform
    // in-plane 3x3 sum of the thread's cells in plane z (4 bits) and the centres
    auto plane_sum = [&](int z, uint32_t (&S)[4], uint32_t &C) {
        uint32_t s0[3], s1[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint32_t *row = buf[z][y - 1 + j];
            const uint32_t a = row[c];
            const uint32_t l = c > 0 ? row[c - 1] : 0u;
            const uint32_t r = c + 1 < DW ? row[c + 1] : 0u;
            const uint32_t L = __builtin_amdgcn_alignbit(a, l, 31);    // cell x-1
            const uint32_t R = __builtin_amdgcn_alignbit(r, a, 1);     // cell x+1
            const uint32_t la = L ^ a;
            s0[j] = la ^ R;
            s1[j] = (L & a) | (R & la);
            if (j == 1) C = a;
        }
        add3_2(s0[0], s1[0], s0[1], s1[1], s0[2], s1[2], S);
    };
    for (int g = 1; g <= gens; ++g) {
        const int z_lo = g, z_hi = W - 1 - g;     // planes (and rows) updated by this generation
        const int steps = (z_hi - z_lo + Sh::NP) / Sh::NP;   // planes per part (uniform)
        const int za = z_lo + part * steps, zb = min(z_hi, za + steps - 1);   // this part's planes
        const bool active = worker && y >= g && y <= W - 1 - g;
        uint32_t Sp[4], Sc[4], Cc = 0u, Cp = 0u, pend = 0u, first = 0u;
        if (active) {
            plane_sum(za - 1, Sp, Cp);
            plane_sum(za, Sc, Cc);
        }
        __syncthreads();   // plane za is read here and rewritten at step za + 1
        for (int i = 0; i < steps; ++i) {
            const int z = za + i;
            if (active && z <= zb) {
                uint32_t Sn[4], Cn;
                plane_sum(z + 1, Sn, Cn);
                if (z > za) {
                    if (part > 0 && z == za + 1) first = pend;   // written at the end
                    else buf[z - 1][y][c] = pend;
                }
                // U = Sp + Sc (5 bits), T = U + Sn (5 bits, at most 27)
                uint32_t u[5], tt[5], cr = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t x1 = Sp[b] ^ Sc[b];
                    u[b] = x1 ^ cr;
                    cr = (Sp[b] & Sc[b]) | (cr & x1);
                }
                u[4] = cr;
                cr = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t x1 = u[b] ^ Sn[b];
                    tt[b] = x1 ^ cr;
                    cr = (u[b] & Sn[b]) | (cr & x1);
                }
                tt[4] = u[4] ^ cr;
                // B6/S567 on the count with the centre: T == 6, or T in {7, 8} and alive
                const uint32_t e67 = ~tt[4] & ~tt[3] & tt[2] & tt[1];
                const uint32_t e8 = ~tt[4] & tt[3] & ~tt[2] & ~tt[1] & ~tt[0];
                uint32_t res = (e67 & (~tt[0] | Cc)) | (Cc & e8);
                if (!interior) {
                    const int32_t gy = ys + y, gz = zs + z;
                    res &= (gy < 0 || gz < 0) ? 0u : ca2k_keep_bits(gx, gy + gz, n);
                }
                pend = res;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    Sp[b] = Sc[b];
                    Sc[b] = Sn[b];
                }
                Cc = Cn;
            }
            if (i & 1) __syncthreads();
        }
        if (steps & 1) __syncthreads();            // (uniform) every step's reads are done
        if (active && za <= zb) {
            buf[zb][y][c] = pend;                   // the part's last new plane
            if (part > 0 && zb > za) buf[za][y][c] = first;
        }
        __syncthreads();
    }

    // 3. Write the tile: 16 cells per lane-step, rho / 16 per tile row.
    constexpr int LPR = RHO / 16;
    for (int q = tid; q < RHO * RHO * LPR; q += NT) {
        const int lc = q % LPR, yy = (q / LPR) % RHO, zz = q / (LPR * RHO);
        const int32_t gy = y0 + yy, gz = z0 + zz, x = x0 + 16 * lc;
        const int32_t v = n - gy - gz - x + 1;
        if (gy + gz > n || v <= 0) continue;
        const int b = KH + 16 * lc;                   // region bit of the first cell
        const uint32_t bits = buf[KH + zz][KH + yy][b / 32] >> (b % 32);
        const uint32_t w0 = unpack4(bits), w1 = unpack4(bits >> 4), w2 = unpack4(bits >> 8),
                       w3 = unpack4(bits >> 12);
        uint8_t *row = out + (int64_t)gz * p2 + (int64_t)gy * p1;
        if (v >= 16) {
            *reinterpret_cast<uint4 *>(row + x) = make_uint4(w0, w1, w2, w3);
        } else {
            const int32_t r = gy + gz;
            st_masked(row, x, r, n, w0);
            st_masked(row, x + 4, r, n, w1);
            st_masked(row, x + 8, r, n, w2);
            st_masked(row, x + 12, r, n, w3);
        }
    }
}

// (the launch bound is Ca3kShape<RHO, KH>::NT, written without commas)
template <int RHO, int KH, bool BB, bool SAFE>
__global__ __launch_bounds__(3 * ((((RHO + 2 * KH) / 32 * (RHO + 2 * KH - 2) + 63) / 64) * 64)) void k_ca3k(
    const Plan P, const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int gens)
{
    static_assert(3 * ((((RHO + 2 * KH) / 32 * (RHO + 2 * KH - 2) + 63) / 64) * 64) == Ca3kShape<RHO, KH>::NT,
                  "launch bound");
    int32_t t[4] = {0, 0, 0, 0};
    const WgId g = wg_id(P);
    if (BB) {
        decode_bb(P, g.x, g.y, g.z, t);
    } else {
        if (!decode_h<3>(P, g.x, t)) return;
    }
    ca3k_tile<RHO, KH, SAFE>(P, in, out, t, gens);
}

}  // namespace smap
