// smap_ca2.hpp -- one step of Life (B3/S23) on Delta_n^2, uint8 cells.
//
// The CA test of Section 5.1 (Table tab:tests) on the 2-simplex; cells
// outside the simplex are dead (the paper's periodic boundary has no meaning
// on a triangle).
//
// Work split.  A workgroup owns a rho x rho tile (from H or BB).  Each lane
// holds 16 consecutive cells of a row in four 32-bit registers (SWAR bytes),
// loaded and stored as one 16-byte access, so a segment of rho/16 lanes
// covers one tile row.  A wave holds 64/(rho/16) segments; every segment
// walks R consecutive rows of the tile downwards,
// keeping the horizontal 3-sums of the previous, current and next rows in
// registers, so every input row is fetched from memory once per segment
// (plus one halo row above and below).  Rows are fetched in blocks of D so
// that D independent loads per wave are in flight: the walk is otherwise a
// chain of dependent row loads and runs at memory latency, not bandwidth.  The left/right neighbour bytes come
// from the adjacent lanes through DPP wave shifts; the two halo bytes of a
// segment come from one extra load by its first and last lane.
//
// Per dword of 4 cells: h = left + centre + right (bytes, <= 3), t = h(y-1) + h(y) +
// h(y+1) (<= 9, the 3x3 sum including the centre), next = (t == 3) |
// (alive & t == 4), evaluated byte-wise with bit-7 tests that cannot carry
// between bytes (see life_b3s23).
//
// Boundary handling is per lane: a lane whose 16 cells are inside loads
// and stores them as one (unaligned; gfx9 global memory accepts unaligned
// accesses) 16-byte access; the lane the hypotenuse cuts zeroes the bytes
// outside after loading (the input there is arbitrary) and stores only the
// cells inside; lanes beyond it touch nothing.  No access ever covers a
// dword without a simplex cell, except the tail bytes of a 16-byte load
// that stays inside the buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_decode.hpp"
#include "smap_point.hpp"

namespace smap {

__device__ __forceinline__ uint32_t ld_u32(const uint8_t *p)
{
    return *reinterpret_cast<const uint32_t *>(p);
}

__device__ __forceinline__ void st_u32(uint8_t *p, uint32_t v)
{
    *reinterpret_cast<uint32_t *>(p) = v;
}

// Cells (row r, columns x..x+3) of a row with pitch `pitch`, cells outside
// { 0 <= x, x + r <= n, 0 <= r <= n } reading as 0.  `r` is the sum of all
// coordinates but x_1 (the row's "height" in the simplex), `row` points at
// column 0 of the row, `total` is the buffer size in bytes minus the row's
// base offset (for the last-row bound).
__device__ __forceinline__ uint32_t ld_masked(const uint8_t *row, int32_t x, int32_t r,
                                              int32_t n, int64_t room)
{
    const int32_t v = n - r - x + 1;          // simplex cells from x on
    if (r < 0 || v <= 0 || x < 0) return 0u;  // (x < 0 only for the left halo at x = -4)
    uint32_t d;
    if ((int64_t)x + 4 <= room) {
        d = ld_u32(row + x);
    } else {                                  // last dword of the buffer (tiny n)
        d = 0u;
        for (int k = 0; k < 4 && k < v; ++k) d |= (uint32_t)row[x + k] << (8 * k);
    }
    return v >= 4 ? d : (d & ((1u << (8 * v)) - 1u));
}

__device__ __forceinline__ void st_masked(uint8_t *row, int32_t x, int32_t r, int32_t n,
                                          uint32_t val)
{
    const int32_t v = n - r - x + 1;
    if (r < 0 || v <= 0) return;
    if (v >= 4) {
        st_u32(row + x, val);
    } else {
        // at most 3 bytes; unrolled (no loop), so every path issues a bounded
        // number of stores and the wait counts before later loads stay exact
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < v) row[x + k] = (uint8_t)(val >> (8 * k));
    }
}

// Life B3/S23 on four byte cells: t = 3x3 sum including the centre (<= 9),
// c = centre (0/1).  next = 1 iff t >= 3 and t - 3 <= c.  With d = t + 0x7D
// per byte, bit 7 of d is (t >= 3); e = d - (c + 1) has bit 7 clear iff
// t - 3 <= c (no byte borrows or carries: 0x7B <= e, d <= 0x86).
__device__ __forceinline__ uint32_t life_b3s23(uint32_t t, uint32_t c)
{
    const uint32_t d = t + 0x7D7D7D7Du;
    const uint32_t e = d - (c + 0x01010101u);
    return ((d & ~e) >> 7) & 0x01010101u;
}

// Sum of left, centre and right neighbours of the 16 cells c[0..3] of a lane
// (c[0] lowest addresses), given the dword just before c[0] (lprev) and the
// dword just after c[3] (rnext).
__device__ __forceinline__ void hsum16(const uint32_t *c, uint32_t lprev, uint32_t rnext, uint32_t *h)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t l = i == 0 ? lprev : c[i - 1];
        const uint32_t r = i == 3 ? rnext : c[i + 1];
        h[i] = __builtin_amdgcn_alignbyte(c[i], l, 3) + c[i] + __builtin_amdgcn_alignbyte(r, c[i], 1);
    }
}

// The neighbouring lanes' boundary dwords (DPP) or, at a segment edge, the
// halo dword e.  Written as value selects: conditional writes through
// references here were turned into a dynamically addressed scratch store.
template <int S>
__device__ __forceinline__ uint32_t lane_prev(const uint32_t *c, uint32_t e, int sl)
{
    const uint32_t d = (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)c[3], 0x138, 0xf, 0xf, false);  // wave_shr:1
    return sl == 0 ? e : d;
}
template <int S>
__device__ __forceinline__ uint32_t lane_next(const uint32_t *c, uint32_t e, int sl)
{
    const uint32_t d = (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)c[0], 0x130, 0xf, 0xf, false);  // wave_shl:1
    return sl == S - 1 ? e : d;
}

// Shape constants of a CA2 tile walk: the W waves of a workgroup stand WX
// side by side along x (each on an RHO/WX-byte column) and W/WX deep along
// y; S lanes per column row, SEGS row segments per wave, SUB sub-blocks
// (workgroups) per tile.
template <int RHO, int W, int R, int WX = 1>
struct Ca2Walk {
    static constexpr int SW = RHO / WX;          // bytes of a wave's column
    static constexpr int S = SW / 16;
    static constexpr int SEGS = 64 / S;
    static constexpr int WY = W / WX;
    static constexpr int SUB = RHO / (WY * SEGS * R);
    static_assert(S >= 2 && S <= 64 && 64 % S == 0 && R >= 1 && SUB >= 1 && W % WX == 0 &&
                  SW * WX == RHO && SUB * WY * SEGS * R == RHO && (SUB & (SUB - 1)) == 0,
                  "bad CA2 tile shape");
};

// One Life step of sub-block `sub` of the rho x rho tile t (workgroup body).
// Each lane holds 16 cells of a row (one unaligned 16-byte access, four SWAR
// dwords); a segment of rho/16 lanes covers a tile row; each segment walks R
// rows.  A tile is split into SUB = rho / (W * SEGS * R) sub-blocks of rows,
// one workgroup each.
template <int RHO, int W, int R, int D, bool SAFE, int WX = 1>
__device__ __forceinline__ void ca2_tile(const Plan &P, const uint8_t *__restrict__ in,
                                         uint8_t *__restrict__ out, const int32_t *t, uint32_t sub)
{
    using Sh = Ca2Walk<RHO, W, R, WX>;
    constexpr int S = Sh::S, SEGS = Sh::SEGS, SW = Sh::SW, WY = Sh::WY;
    const int32_t n = P.n;
    const int32_t xt = t[0] * RHO, y0 = t[1] * RHO + (int32_t)sub * (WY * SEGS * R);
    if (xt + y0 > n) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // scalar
    const int seg = lane / S, sl = lane % S;
    const int32_t x0 = xt + (wave % WX) * SW;     // the wave's column
    const int32_t ywave = y0 + (wave / WX) * SEGS * R;   // first row of the wave's first segment
    // rows after n - x0 hold no simplex cell in this tile column (wave-uniform)
    const int32_t rows = min(R, n - x0 - ywave + 1);
    if (rows <= 0) return;                          // whole wave idle (no barriers here)

    const int64_t pitch = P.stride[1];
    const int64_t total = pitch * pitch;
    const int32_t x = x0 + 16 * sl;
    const int32_t xe = (sl == 0) ? x0 - 4 : x0 + SW;
    const bool is_edge = (sl == 0) || (sl == S - 1);
    // Row r of the wave (r = -1 .. R) is addressed as a wave-uniform row
    // pointer (scalar) plus a per-lane 32-bit offset that is the same for
    // every row: the segment's row offset plus the column.  The halo offset
    // of a lane that never loads it is clamped to 0 (offsets are unsigned).
    const uint32_t seg_off = (uint32_t)(seg * R) * (uint32_t)pitch;
    const uint32_t off_c = seg_off + (uint32_t)x;
    const uint32_t off_e = seg_off + (uint32_t)max(xe, 0);
    const int32_t lane_rows = seg * R;             // the lane's row is ywave + r + lane_rows

    // Rows with a simplex cell in this lane: 0 <= y <= n and x <= n - y.
    // For n >= 15 a 16-byte access starting at such a cell never passes the
    // end of the buffer (worst case y = n, x = 0: n (n+1) + 16 <= (n+1)^2),
    // and neither does the 4-byte halo access; the host launches the SAFE
    // instantiation (byte-safe loads through ld_masked) for smaller n.

    // Raw loads of wave row r: the lane's 16 cells and its halo dword (first
    // and last lane of a segment).  No masking here, so the loads of a block
    // issue back to back.  The 16-byte load is issued by every lane, reading
    // the buffer's first 16 bytes when the lane has no simplex cell in the
    // row (mask_row clears it): unconditional loads keep the number of loads
    // issued after a row known, so the wait before the row's use covers that
    // row only and the loads of the next block stay in flight.  The halo load
    // (few lanes) is conditional and issued first.
    auto load_raw = [&](int32_t r, uint32_t *c, uint32_t &e) {
        const int32_t y = ywave + r + lane_rows;
        const bool yin = (uint32_t)y <= (uint32_t)n;   // 0 <= y <= n
        const uint8_t *rowp = in + (int64_t)(ywave + r) * pitch;   // wave-uniform
        // rows past r = rows (the halo below the last output row) are
        // never needed: their loads read the buffer's first bytes instead
        const bool need = yin && r <= rows;            // r <= rows is wave-uniform
        e = 0u;
        if (is_edge && need && xe >= 0 && xe <= n - y) e = ld_u32(rowp + off_e);
        const bool has = need && x <= n - y;
        const uint4 q = *reinterpret_cast<const uint4 *>(has ? rowp + off_c : in);
        c[0] = q.x; c[1] = q.y; c[2] = q.z; c[3] = q.w;
    };
    // Zero the cells of wave row r that lie outside the simplex (only the
    // lane the hypotenuse cuts, and the right halo byte, can hold any).
    auto mask_row = [&](int32_t r, uint32_t *c, uint32_t &e) {
        const int32_t y = ywave + r + lane_rows;
        const int32_t v = y < 0 ? 0 : n - y - x + 1;  // simplex cells from x on
        if (v < 16) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t keep = v - 4 * i;
                c[i] = keep >= 4 ? c[i] : (keep <= 0 ? 0u : c[i] & ((1u << (8 * keep)) - 1u));
            }
        }
        const int32_t ve = n - y - xe + 1;
        if (ve < 4) e = ve <= 0 ? 0u : e & ((1u << (8 * ve)) - 1u);
    };
    // Byte-safe load of wave row r for tiny n.
    auto load_safe = [&](int32_t r, uint32_t *c, uint32_t &e) {
        c[0] = c[1] = c[2] = c[3] = 0u;
        e = 0u;
        const int32_t y = ywave + r + lane_rows;
        if ((uint32_t)y > (uint32_t)n) return;
        const int64_t rb = (int64_t)y * pitch;
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = ld_masked(in + rb, x + 4 * i, y, n, total - rb);
        if (is_edge) e = ld_masked(in + rb, xe, y, n, total - rb);
    };
    auto store_row = [&](int32_t r, const uint32_t *res) {
        const int32_t y = ywave + r + lane_rows;
        if ((uint32_t)y > (uint32_t)n) return;
        const int32_t v = n - y - x + 1;
        if (v <= 0) return;
        if (v >= 16) {
            uint8_t *rowp = out + (int64_t)(ywave + r) * pitch;    // wave-uniform
            *reinterpret_cast<uint4 *>(rowp + off_c) = make_uint4(res[0], res[1], res[2], res[3]);
        } else {
            uint8_t *row = out + (int64_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 4; ++i) st_masked(row, x + 4 * i, y, n, res[i]);
        }
    };
    auto load_row = [&](int32_t r, uint32_t *c, uint32_t &e) {
        if constexpr (SAFE) {
            load_safe(r, c, e);
        } else {
            load_raw(r, c, e);
            mask_row(r, c, e);
        }
    };

    // Prologue: the row above the segment and its first row.
    uint32_t hp[4], hc[4], cc[4];
    {
        uint32_t ca[4], ea, eb;
        load_row(-1, ca, ea);
        load_row(0, cc, eb);
        hsum16(ca, lane_prev<S>(ca, ea, sl), lane_next<S>(ca, ea, sl), hp);
        hsum16(cc, lane_prev<S>(cc, eb, sl), lane_next<S>(cc, eb, sl), hc);
    }

    // Blocks of D output rows; block r0 needs rows r0+1 .. r0+D.  The loads
    // of the next block are issued before the current block is summed, into
    // the other of two register sets (the loop is unrolled by two, so no
    // register copy waits for a load).  `rows` is wave-uniform, so the
    // guards are scalar branches.
    auto load_block = [&](int32_t r0, uint32_t (&c)[D][4], uint32_t (&e)[D]) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if constexpr (SAFE) load_safe(r0 + 1 + k, c[k], e[k]);
            else load_raw(r0 + 1 + k, c[k], e[k]);
        }
    };
    auto sum_block = [&](int32_t r0, uint32_t (&c)[D][4], uint32_t (&e)[D]) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if constexpr (!SAFE) mask_row(r0 + 1 + k, c[k], e[k]);
            if (r0 + 1 + k > rows) {  // below the segment's last needed row
                c[k][0] = c[k][1] = c[k][2] = c[k][3] = 0u;
                e[k] = 0u;
            }
            uint32_t hn[4], res[4];
            hsum16(c[k], lane_prev<S>(c[k], e[k], sl), lane_next<S>(c[k], e[k], sl), hn);
#pragma unroll
            for (int i = 0; i < 4; ++i) res[i] = life_b3s23(hp[i] + hc[i] + hn[i], cc[i]);
            if (r0 + k < rows) store_row(r0 + k, res);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                hp[i] = hc[i];
                hc[i] = hn[i];
                cc[i] = c[k][i];
            }
        }
    };
    // Both halves of the unrolled loop always run (rows past the segment's
    // last are cleared and not stored), so every block issues its loads.
    uint32_t cA[D][4], eA[D], cB[D][4], eB[D];
    load_block(0, cA, eA);
    for (int32_t r0 = 0; r0 < rows; r0 += 2 * D) {
        load_block(r0 + D, cB, eB);
        sum_block(r0, cA, eA);
        load_block(r0 + 2 * D, cA, eA);
        sum_block(r0 + D, cB, eB);
    }
}

// The CA2 kernel: the launch grid is the map's grid times SUB (sub-blocks of
// a tile adjacent in H, the y grid coordinate in BB).
template <int RHO, int W, int R, int D, bool BB, bool SAFE, int WX = 1>
__global__ __launch_bounds__(64 * W) void k_ca2(const Plan P, const uint8_t *__restrict__ in,
                                                uint8_t *__restrict__ out)
{
    constexpr int SUB = Ca2Walk<RHO, W, R, WX>::SUB;
    int32_t t[4] = {0, 0, 0, 0};
    uint32_t sub;
    const WgId g = wg_id(P);
    if (BB) {
        decode_bb(P, g.x, g.y / SUB, 0, t);
        sub = g.y % SUB;
    } else {
        if (!decode_h<2>(P, g.x / SUB, t)) return;
        sub = g.x % SUB;
    }
    ca2_tile<RHO, W, R, D, SAFE, WX>(P, in, out, t, sub);
}

}  // namespace smap
