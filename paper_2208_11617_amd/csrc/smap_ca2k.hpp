// smap_ca2k.hpp -- several Life generations (B3/S23) per pass over HBM.
//
// The paper's automaton test runs a fixed number of steps (Section 5.1).
// One launch here advances every cell of Delta_n^2 by `gens` <= KH
// generations: a workgroup loads its rho x rho tile plus a halo of KH cells
// on each side into LDS (cells outside the simplex, or outside the box, are
// dead), steps the whole region `gens` times in LDS, and writes the tile.
// Each generation the band of cells whose neighbourhood reached outside the
// loaded region grows inward by one, so after gens <= KH generations the
// tile itself is exact.  HBM traffic per generation drops from 2 bytes per
// cell to about ((rho + 2 KH)^2 / rho^2 + 1) / gens.
//
// In LDS a cell is one bit: two buffers of (rho + 2 KH) rows x
// (rho + 2 KH) / 32 dwords; bit b of dword c of row r is the cell
// x = x0 - KH + 32c + b, y = y0 - KH + r.  The neighbour count is
// bit-sliced: the horizontal 3-sum of a row is a 2-bit number per cell
// (a full adder over the row and its copies shifted by one cell, the
// shifts funnelled across dword boundaries), the 3x3 sum including the
// centre is the sum of three such numbers (4 bits, at most 9), and the rule
// is a few logic operations on those bits: 32 cells per operation.  A
// thread owns one dword column and a run of rows and walks the run with the
// horizontal sums of the two previous rows in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_decode.hpp"

namespace smap {

template <int RHO, int KH>
struct Ca2kShape {
    static constexpr int W = RHO + 2 * KH;   // cells per staged row (and rows)
    static constexpr int DW = W / 32;         // dwords (32 cells) per staged row
    static constexpr int NT = W <= 160 ? 64 : 256;   // threads
    static constexpr int SEGS = NT / DW;      // row runs per dword column
    static constexpr int RUN = (W + SEGS - 1) / SEGS;
    static_assert(KH % 16 == 0 && RHO % 32 == 0 && W % 32 == 0 && DW <= NT, "bad CA2K shape");
};

// Simplex cells of the dword (x .. x+3, y): bytes kept.
__device__ __forceinline__ uint32_t ca2k_keep_mask(int32_t x, int32_t y, int32_t n)
{
    if (x < 0 || y < 0) return 0u;
    const int32_t keep = n - y - x + 1;
    return keep >= 4 ? 0xFFFFFFFFu : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
}

// Simplex cells of the 32 cells x .. x+31 of row y, as bits (cells left of
// the box, x < 0, and past the hypotenuse cleared).
__device__ __forceinline__ uint32_t ca2k_keep_bits(int32_t x, int32_t y, int32_t n)
{
    if (y < 0 || x <= -32) return 0u;
    const int32_t hi = n - y - x + 1;               // cells x .. x+hi-1 satisfy x + y <= n
    uint32_t m = hi >= 32 ? 0xFFFFFFFFu : (hi <= 0 ? 0u : (1u << hi) - 1u);
    if (x < 0) m &= 0xFFFFFFFFu << (-x);            // the low -x cells are left of the box
    return m;
}

// Four 0/1 bytes -> 4 bits (byte k -> bit k): the product places byte k's
// bit at bit 24 + k, every other partial product lands on a distinct bit
// below 24 or beyond bit 31, so nothing carries into bits 24..27.
__device__ __forceinline__ uint32_t pack4(uint32_t d) { return ((d * 0x01020408u) >> 24) & 0xFu; }

// 4 bits -> four 0/1 bytes (bit k -> byte k): bit k of v times 2^(7j)
// lands on bit k + 7j, a multiple of 8 only for j = k, with no carries.
__device__ __forceinline__ uint32_t unpack4(uint32_t v) { return ((v & 0xFu) * 0x00204081u) & 0x01010101u; }

template <int RHO, int KH, bool SAFE>
__device__ __forceinline__ void ca2k_tile(const Plan &P, const uint8_t *__restrict__ in,
                                          uint8_t *__restrict__ out, const int32_t *t, int gens)
{
    using Sh = Ca2kShape<RHO, KH>;
    constexpr int W = Sh::W, DW = Sh::DW, NT = Sh::NT, RUN = Sh::RUN;
    __shared__ uint32_t buf[2][W][DW];
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO, y0 = t[1] * RHO;
    if (x0 + y0 > n) return;                    // uniform: BB tile outside the simplex
    const int64_t pitch = P.stride[1];
    const int64_t total = pitch * pitch;
    const int tid = threadIdx.x;
    const int32_t xs = x0 - KH, ys = y0 - KH;   // cell of bit 0 of dword 0 of row 0

    // 1. Stage the region: each dword is two 16-byte chunks, loaded from
    //    their first cell (x >= 0 for every chunk with a simplex cell, KH
    //    being a multiple of 16), cleared outside the simplex, packed to bits.
    for (int q = tid; q < W * DW; q += NT) {
        const int r = q / DW, c = q % DW;
        const int32_t y = ys + r;
        uint32_t word = 0u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t x = xs + 32 * c + 16 * h;
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            const bool has = y >= 0 && y <= n && x >= 0 && x <= n - y;
            if constexpr (SAFE) {
                if (has) {
                    const int64_t rb = (int64_t)y * pitch;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w[i] = ld_masked(in + rb, x + 4 * i, y, n, total - rb);
                }
            } else {
                const uint4 v = *reinterpret_cast<const uint4 *>(has ? in + (int64_t)y * pitch + x : in);
                w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] &= ca2k_keep_mask(x + 4 * i, y, n);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) word |= pack4(w[i]) << (16 * h + 4 * i);
        }
        buf[0][r][c] = word;
    }
    __syncthreads();

    // 2. `gens` generations, buffer g & 1 -> (g + 1) & 1.  Generation g
    //    (0-based) only needs rows g+1 .. W-2-g (the cells nearer the
    //    region's edge are already stale).  A workgroup whose whole region
    //    lies inside the simplex skips the simplex mask.
    const int col = tid % DW, seg = tid / DW;
    const bool worker = tid < Sh::SEGS * DW;
    const int r_a = seg * RUN, r_b = min(W, r_a + RUN);
    const int32_t xcol = xs + 32 * col;
    const bool interior = xs >= 0 && ys >= 0 && xs + ys + 2 * (W - 1) <= n;   // uniform
    for (int g = 0; g < gens; ++g) {
        const uint32_t(*src)[DW] = buf[g & 1];
        uint32_t(*dst)[DW] = buf[(g + 1) & 1];
        const int lo = max(r_a, g + 1), hi = min(r_b, W - 1 - g);
        if (worker && lo < hi) {
            // horizontal 3-sum of row r as two bit planes (s0: bit 0, s1: bit 1)
            auto hrow = [&](int r, uint32_t &s0, uint32_t &s1, uint32_t &a) {
                a = src[r][col];
                const uint32_t l = col > 0 ? src[r][col - 1] : 0u;
                const uint32_t rr = col + 1 < DW ? src[r][col + 1] : 0u;
                const uint32_t L = __builtin_amdgcn_alignbit(a, l, 31);    // cell x-1
                const uint32_t R = __builtin_amdgcn_alignbit(rr, a, 1);    // cell x+1
                const uint32_t la = L ^ a;
                s0 = la ^ R;
                s1 = (L & a) | (R & la);
            };
            uint32_t p0, p1, c0, c1, n0, n1, pa, ca, na;
            hrow(lo - 1, p0, p1, pa);
            hrow(lo, c0, c1, ca);
            for (int r = lo; r < hi; ++r) {
                hrow(r + 1, n0, n1, na);
                // T = p + c + n (three 2-bit numbers) as bits q3 q2 q1 q0
                const uint32_t t0 = p0 ^ c0, k0 = p0 & c0;
                const uint32_t x1 = p1 ^ c1;
                const uint32_t t1 = x1 ^ k0, k1 = (p1 & c1) | (k0 & x1);
                const uint32_t q0 = t0 ^ n0, m0 = t0 & n0;
                const uint32_t y1 = t1 ^ n1;
                const uint32_t q1 = y1 ^ m0, m1 = (t1 & n1) | (m0 & y1);
                const uint32_t q2 = k1 ^ m1, q3 = k1 & m1;
                // B3/S23 on the count with the centre: T == 3, or T == 4 and alive
                uint32_t res = ~q3 & ((q0 & q1 & ~q2) | (ca & ~q0 & ~q1 & q2));
                if (!interior) res &= ca2k_keep_bits(xcol, ys + r, n);
                dst[r][col] = res;
                p0 = c0; p1 = c1;
                c0 = n0; c1 = n1;
                ca = na;
            }
        }
        __syncthreads();
    }

    // 3. Write the tile: 16 cells per lane-step, rho / 16 per tile row.
    const uint32_t(*fin)[DW] = buf[gens & 1];
    constexpr int LPR = RHO / 16;
    for (int q = tid; q < RHO * LPR; q += NT) {
        const int rr = q / LPR, lc = q % LPR;
        const int32_t y = y0 + rr, x = x0 + 16 * lc;
        const int32_t v = n - y - x + 1;
        if (y > n || v <= 0) continue;
        const int b = KH + 16 * lc;                   // region bit of the first cell
        const uint32_t bits = fin[KH + rr][b / 32] >> (b % 32);
        const uint32_t w0 = unpack4(bits), w1 = unpack4(bits >> 4), w2 = unpack4(bits >> 8),
                       w3 = unpack4(bits >> 12);
        uint8_t *row = out + (int64_t)y * pitch;
        if (v >= 16) {
            *reinterpret_cast<uint4 *>(row + x) = make_uint4(w0, w1, w2, w3);
        } else {
            st_masked(row, x, y, n, w0);
            st_masked(row, x + 4, y, n, w1);
            st_masked(row, x + 8, y, n, w2);
            st_masked(row, x + 12, y, n, w3);
        }
    }
}

// (the launch bound is Ca2kShape<RHO, KH>::NT, written without commas)
template <int RHO, int KH, bool BB, bool SAFE>
__global__ __launch_bounds__(RHO + 2 * KH <= 160 ? 64 : 256) void k_ca2k(const Plan P, const uint8_t *__restrict__ in,
                                                                        uint8_t *__restrict__ out, int gens)
{
    static_assert(Ca2kShape<RHO, KH>::NT == (RHO + 2 * KH <= 160 ? 64 : 256), "launch bound");
    int32_t t[4] = {0, 0, 0, 0};
    const WgId g = wg_id(P);
    if (BB) {
        decode_bb(P, g.x, g.y, 0, t);
    } else {
        if (!decode_h<2>(P, g.x, t)) return;
    }
    ca2k_tile<RHO, KH, SAFE>(P, in, out, t, gens);
}

}  // namespace smap
