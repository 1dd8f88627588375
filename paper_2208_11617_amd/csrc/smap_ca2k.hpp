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
// LDS layout: two buffers of (rho + 2 KH) rows x (rho + 2 KH) / 4 dwords;
// byte b of dword c of row r is the cell x = x0 - KH + 4c + b,
// y = y0 - KH + r.  A thread owns a pair of dword columns and a run of rows
// and walks it with the horizontal 3-sums of the previous two rows in
// registers; left/right neighbour bytes come from the adjacent dwords
// (`alignbyte`), the dwords beyond the region read as dead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_decode.hpp"

namespace smap {

template <int RHO, int KH>
struct Ca2kShape {
    static constexpr int W = RHO + 2 * KH;   // cells per staged row (and rows)
    static constexpr int DW = W / 4;          // dwords per staged row
    static constexpr int PC = DW / 2;         // dword pairs per row (a thread's column)
    static constexpr int NT = 256;            // threads
    static constexpr int SEGS = NT / PC;      // row runs per column
    static constexpr int RUN = (W + SEGS - 1) / SEGS;
    static_assert(KH % 16 == 0 && RHO % 16 == 0 && PC <= NT, "bad CA2K shape");
};

// Simplex cells of the dword at (x .. x+3, y): bytes kept.
__device__ __forceinline__ uint32_t ca2k_keep_mask(int32_t x, int32_t y, int32_t n)
{
    if (x < 0 || y < 0) return 0u;
    const int32_t keep = n - y - x + 1;
    return keep >= 4 ? 0xFFFFFFFFu : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
}

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
    const int32_t xs = x0 - KH, ys = y0 - KH;   // cell of byte 0 of dword 0 of row 0

    // 1. Stage the region: 16-byte chunks (W / 16 per row), loaded from the
    //    first simplex cell of the chunk (x >= 0 for every chunk that has one,
    //    since KH is a multiple of 16), cleared outside the simplex.
    constexpr int CPR = W / 16, NCH = W * CPR;
    for (int q = tid; q < NCH; q += NT) {
        const int r = q / CPR, c = q % CPR;
        const int32_t y = ys + r, x = xs + 16 * c;
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
        for (int i = 0; i < 4; ++i) buf[0][r][4 * c + i] = w[i];
    }
    __syncthreads();

    // 2. `gens` generations, buffer g & 1 -> (g + 1) & 1.  A thread owns a
    //    pair of dword columns (8 cells) and a run of rows.  Generation g
    //    (0-based) only needs rows g+1 .. W-2-g (the cells nearer the region's
    //    edge are already invalid).  A workgroup whose whole region lies
    //    inside the simplex skips the simplex mask.
    const int pc = tid % Sh::PC, seg = tid / Sh::PC;
    const bool worker = tid < Sh::SEGS * Sh::PC;
    const int r_a = seg * RUN, r_b = min(W, r_a + RUN);
    const int c0 = 2 * pc;                     // first of the thread's two dwords
    const int32_t xcol = xs + 4 * c0;
    const bool interior = xs >= 0 && ys >= 0 && xs + ys + 2 * (W - 1) <= n;   // uniform
    for (int g = 0; g < gens; ++g) {
        const uint32_t(*src)[DW] = buf[g & 1];
        uint32_t(*dst)[DW] = buf[(g + 1) & 1];
        const int lo = max(r_a, g + 1), hi = min(r_b, W - 1 - g);
        if (worker && lo < hi) {
            // horizontal 3-sums of the pair in row r, and its centre cells
            auto hrow = [&](int r, uint32_t &h0, uint32_t &h1, uint32_t &m0, uint32_t &m1) {
                const uint2 cc = *reinterpret_cast<const uint2 *>(&src[r][c0]);
                const uint32_t l = c0 > 0 ? src[r][c0 - 1] : 0u;
                const uint32_t rr = c0 + 2 < DW ? src[r][c0 + 2] : 0u;
                m0 = cc.x;
                m1 = cc.y;
                h0 = __builtin_amdgcn_alignbyte(cc.x, l, 3) + cc.x + __builtin_amdgcn_alignbyte(cc.y, cc.x, 1);
                h1 = __builtin_amdgcn_alignbyte(cc.y, cc.x, 3) + cc.y + __builtin_amdgcn_alignbyte(rr, cc.y, 1);
            };
            uint32_t hp0, hp1, hc0, hc1, cc0, cc1, d0, d1;
            hrow(lo - 1, hp0, hp1, d0, d1);
            hrow(lo, hc0, hc1, cc0, cc1);
            for (int r = lo; r < hi; ++r) {
                uint32_t hn0, hn1, cn0, cn1;
                hrow(r + 1, hn0, hn1, cn0, cn1);
                uint32_t res0 = life_b3s23(hp0 + hc0 + hn0, cc0);
                uint32_t res1 = life_b3s23(hp1 + hc1 + hn1, cc1);
                if (!interior) {
                    res0 &= ca2k_keep_mask(xcol, ys + r, n);
                    res1 &= ca2k_keep_mask(xcol + 4, ys + r, n);
                }
                *reinterpret_cast<uint2 *>(&dst[r][c0]) = make_uint2(res0, res1);
                hp0 = hc0; hp1 = hc1;
                hc0 = hn0; hc1 = hn1;
                cc0 = cn0; cc1 = cn1;
            }
        }
        __syncthreads();
    }

    // 3. Write the tile: 16 cells per lane, rho / 16 lanes per tile row.
    const uint32_t(*fin)[DW] = buf[gens & 1];
    constexpr int LPR = RHO / 16;
    for (int q = tid; q < RHO * LPR; q += NT) {
        const int rr = q / LPR, lc = q % LPR;
        const int32_t y = y0 + rr, x = x0 + 16 * lc;
        const int32_t v = n - y - x + 1;
        if (y > n || v <= 0) continue;
        const int r = rr + KH, c = (KH + 16 * lc) / 4;
        const uint32_t w0 = fin[r][c], w1 = fin[r][c + 1], w2 = fin[r][c + 2], w3 = fin[r][c + 3];
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

template <int RHO, int KH, bool BB, bool SAFE>
__global__ __launch_bounds__(256) void k_ca2k(const Plan P, const uint8_t *__restrict__ in,
                                              uint8_t *__restrict__ out, int gens)
{
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
