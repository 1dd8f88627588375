// smap_ca2.hpp -- one step of Life (B3/S23) on Delta_n^2, uint8 cells.
//
// The CA test of Section 5.1 (Table tab:tests) on the 2-simplex; cells
// outside the simplex are dead (the paper's periodic boundary has no meaning
// on a triangle).
//
// Work split.  A workgroup owns a rho x rho tile (from H or BB).  Each lane
// holds 4 consecutive cells of a row in one 32-bit register (SWAR bytes), so
// a segment of rho/4 lanes covers one tile row.  A wave holds 64/(rho/4)
// segments; every segment walks R consecutive rows of the tile downwards,
// keeping the horizontal 3-sums of the previous, current and next rows in
// registers, so every input row is fetched from memory once per segment
// (plus one halo row above and below).  The left/right neighbour bytes come
// from the adjacent lanes through DPP wave shifts; the two halo bytes of a
// segment come from one extra load by its first and last lane.
//
// Per 4 cells: h = left + centre + right (bytes, <= 3), t = h(y-1) + h(y) +
// h(y+1) (<= 9, the 3x3 sum including the centre), next = (t == 3) |
// (alive & t == 4).  Byte-wise equality uses ((t ^ k) + 0x7F) & 0x80, which
// cannot carry between bytes because every byte is below 0x80.
//
// Boundary handling.  Rows whose whole segment (with halo) lies inside the
// simplex load and store plain dwords.  Other rows zero the cells outside
// the simplex or the box after loading (the input there is arbitrary),
// never load a dword that holds no simplex cell, and store only the cells
// inside (byte stores for the last partial dword).  Rows are unaligned
// (pitch n+1); gfx9 global loads and stores accept unaligned dwords.
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
        for (int k = 0; k < v; ++k) row[x + k] = (uint8_t)(val >> (8 * k));
    }
}

// Life B3/S23 on four byte cells: t = 3x3 sum including the centre.
__device__ __forceinline__ uint32_t life_b3s23(uint32_t t, uint32_t c)
{
    const uint32_t ne3 = (t ^ 0x03030303u) + 0x7F7F7F7Fu;  // bit 7 set where t != 3
    const uint32_t ne4 = (t ^ 0x04040404u) + 0x7F7F7F7Fu;  // bit 7 set where t != 4
    return ((~ne3 | (~ne4 & (c << 7))) >> 7) & 0x01010101u;
}

// left + centre + right neighbours, bytewise, from the lane's dword c, the
// adjacent lanes' dwords (DPP) and the segment's halo dword e.
template <int S>
__device__ __forceinline__ uint32_t hsum3(uint32_t c, uint32_t e, int sl)
{
    uint32_t l = (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)c, 0x138, 0xf, 0xf, false);  // wave_shr:1
    uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)c, 0x130, 0xf, 0xf, false);  // wave_shl:1
    if (sl == 0) l = e;
    if (sl == S - 1) r = e;
    return __builtin_amdgcn_alignbyte(c, l, 3) + c + __builtin_amdgcn_alignbyte(r, c, 1);
}

template <int RHO, int W, bool BB>
__global__ __launch_bounds__(64 * W) void k_ca2(const Plan P, const uint8_t *__restrict__ in,
                                                uint8_t *__restrict__ out)
{
    constexpr int S = RHO / 4;         // lanes per tile row
    constexpr int SEGS = 64 / S;       // row segments per wave
    constexpr int R = RHO / (W * SEGS);  // rows walked by each segment
    static_assert(S >= 2 && S <= 64 && 64 % S == 0 && R >= 1, "bad CA2 tile shape");

    int32_t t[4] = {0, 0, 0, 0};
    if (!wg_tile<2, BB>(P, t)) return;
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO, y0 = t[1] * RHO;
    if (x0 + y0 > n) return;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int seg = lane / S, sl = lane % S;
    const int32_t ywave = y0 + wave * SEGS * R;   // first row of the wave's first segment
    const int32_t ybeg = ywave + seg * R;          // first row of this lane's segment
    // rows after n - x0 hold no simplex cell in this tile column
    const int32_t rows = min(R, n - x0 - ywave + 1);
    if (rows <= 0) return;                          // whole wave idle (no barriers here)

    const int64_t pitch = P.stride[1];
    const int64_t total = pitch * pitch;
    const int32_t x = x0 + 4 * sl;
    const bool has_e = (sl == 0) || (sl == S - 1);
    const int32_t xe = (sl == 0) ? x0 - 4 : x0 + RHO;
    const bool left_ok = x0 >= 4;

    // Load row y of this segment: own dword and (first/last lane) halo dword.
    // `fast` is wave-uniform: every row the wave touches at this step lies
    // inside the simplex with its halo.
    auto load_row = [&](int32_t y, bool fast, uint32_t &c, uint32_t &e) {
        const int64_t rb = (int64_t)y * pitch;
        if (fast) {
            c = ld_u32(in + rb + x);
            e = has_e ? ld_u32(in + rb + xe) : 0u;
        } else {
            const bool yin = (y >= 0) && (y <= n);
            const uint8_t *row = in + (yin ? rb : 0);
            const int64_t room = total - (yin ? rb : 0);
            c = yin ? ld_masked(row, x, y, n, room) : 0u;
            e = (yin && has_e) ? ld_masked(row, xe, y, n, room) : 0u;
        }
    };
    auto fast_at = [&](int32_t r) {  // rows ywave + r + seg * R for all segments
        const int32_t ylo = ywave + r, yhi = ywave + (SEGS - 1) * R + r;
        return left_ok && ylo >= 0 && (x0 + RHO + yhi <= n);
    };

    uint32_t ca, ea, cb, eb, cn, en;
    load_row(ybeg - 1, fast_at(-1), ca, ea);
    load_row(ybeg, fast_at(0), cb, eb);
    load_row(ybeg + 1, fast_at(1), cn, en);
    uint32_t hp = hsum3<S>(ca, ea, sl);
    uint32_t hc = hsum3<S>(cb, eb, sl);
    uint32_t cc = cb;

    for (int32_t r = 0; r < rows; ++r) {
        uint32_t cnn = 0u, enn = 0u;
        if (r + 2 <= rows) load_row(ybeg + r + 2, fast_at(r + 2), cnn, enn);
        const uint32_t hn = hsum3<S>(cn, en, sl);
        const uint32_t res = life_b3s23(hp + hc + hn, cc);
        const int32_t y = ybeg + r;
        if (fast_at(r)) {
            st_u32(out + (int64_t)y * pitch + x, res);
        } else if (y <= n) {
            st_masked(out + (int64_t)y * pitch, x, y, n, res);
        }
        hp = hc;
        hc = hn;
        cc = cn;
        cn = cnn;
        en = enn;
    }
}

}  // namespace smap
