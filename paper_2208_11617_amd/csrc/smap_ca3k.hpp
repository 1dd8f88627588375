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
// LDS: ONE buffer of W = rho + 2 KH planes x W rows x W/4 dwords (64,000
// bytes for rho = 32, KH = 4: two workgroups fit a compute unit).  Byte b of
// dword c of row y of plane z is the cell (x0 - KH + 4c + b, y0 - KH + y,
// z0 - KH + z).  A generation updates the region in place: a thread owns a
// dword column c and RL consecutive rows and walks the planes along z,
// holding the in-plane 3x3 sums of its rows for the two previous planes in
// registers; the new plane z is written one step later, once every thread
// has read the old plane z (one barrier per two planes).  Generation g
// updates planes g .. W-1-g (the only ones still needed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smap_ca2.hpp"
#include "smap_ca3.hpp"
#include "smap_decode.hpp"

namespace smap {

template <int RHO, int KH, int RL>
struct Ca3kShape {
    static constexpr int W = RHO + 2 * KH;        // cells per staged row; rows; planes
    static constexpr int DW = W / 4;               // dwords per staged row
    static constexpr int RG = (W - 2) / RL;        // row groups over rows 1 .. W-2
    static constexpr int NCOL = DW * RG;           // thread columns (dword, row group)
    static constexpr int NT = ((NCOL + 63) / 64) * 64;
    static_assert(W % 4 == 0 && KH % 4 == 0 && RHO % 16 == 0 && (W - 2) % RL == 0 && NT <= 1024,
                  "bad CA3K shape");
};

// Simplex cells of the dword (x .. x+3, y, z): bytes kept.
__device__ __forceinline__ uint32_t ca3k_keep_mask(int32_t x, int32_t y, int32_t z, int32_t n)
{
    if (x < 0 || y < 0 || z < 0) return 0u;
    const int32_t keep = n - z - y - x + 1;
    return keep >= 4 ? 0xFFFFFFFFu : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
}

template <int RHO, int KH, int RL>
__device__ __forceinline__ void ca3k_tile(const Plan &P, const uint8_t *__restrict__ in,
                                          uint8_t *__restrict__ out, const int32_t *t, int gens)
{
    using Sh = Ca3kShape<RHO, KH, RL>;
    constexpr int W = Sh::W, DW = Sh::DW, NT = Sh::NT;
    __shared__ uint32_t buf[W][W][DW];
    const int32_t n = P.n;
    const int32_t x0 = t[0] * RHO, y0 = t[1] * RHO, z0 = t[2] * RHO;
    if (x0 + y0 + z0 > n) return;                // uniform: BB tile outside the simplex
    const int64_t p1 = P.stride[1], p2 = P.stride[2];
    const int64_t total = p2 * p1;
    const int tid = threadIdx.x;
    const int32_t xs = x0 - KH, ys = y0 - KH, zs = z0 - KH;   // cell of byte 0, dword 0, row 0, plane 0

    // 1. Stage the region, dword by dword; cells outside the simplex or the
    //    box read as dead.  From n = 3 on, a dword with a simplex cell can be
    //    read whole (its bytes past the row's simplex part are still inside
    //    the buffer), so LB loads per thread are issued unconditionally (the
    //    buffer's first dword for a dword without one) before any is used.
    constexpr int NL = W * W * DW, LB = 8;
    uint32_t *flat = &buf[0][0][0];
    if (n >= 3) {
        for (int q0 = tid; q0 < NL; q0 += NT * LB) {
            uint32_t v[LB];
#pragma unroll
            for (int k = 0; k < LB; ++k) {
                const int q = min(q0 + k * NT, NL - 1);
                const int c = q % DW, y = (q / DW) % W, z = q / (DW * W);
                const int32_t gx = xs + 4 * c, gy = ys + y, gz = zs + z;
                const uint32_t keep = ca3k_keep_mask(gx, gy, gz, n);
                const uint8_t *a = keep ? in + ((int64_t)gz * p2 + (int64_t)gy * p1 + gx) : in;
                v[k] = ld_u32(a) & keep;
            }
#pragma unroll
            for (int k = 0; k < LB; ++k)
                if (q0 + k * NT < NL) flat[q0 + k * NT] = v[k];
        }
    } else {
        for (int q = tid; q < NL; q += NT) {   // masked loads never read past the buffer
            const int c = q % DW, y = (q / DW) % W, z = q / (DW * W);
            const int32_t gx = xs + 4 * c, gy = ys + y, gz = zs + z;
            uint32_t v = 0u;
            if (gy >= 0 && gz >= 0) {
                const int64_t rb = (int64_t)gz * p2 + (int64_t)gy * p1;
                if (gy + gz <= n) v = ld_masked(in + rb, gx, gy + gz, n, total - rb);
            }
            flat[q] = v;
        }
    }
    __syncthreads();

    // 2. Generations.  Thread column: dword c, rows yb .. yb+RL-1.
    const bool worker = tid < Sh::NCOL;
    const int c = tid % DW;
    const int yb = 1 + RL * (tid / DW);
    const int32_t gx = xs + 4 * c;
    const bool interior = xs >= 0 && ys >= 0 && zs >= 0 && xs + ys + zs + 3 * (W - 1) <= n;   // uniform
    // in-plane 3x3 sums S of the thread's rows in plane z, and their centres
    auto plane_sums = [&](int z, uint32_t (&S)[RL], uint32_t (&C)[RL]) {
        uint32_t h[RL + 2];
#pragma unroll
        for (int j = 0; j < RL + 2; ++j) {
            const uint32_t *row = buf[z][yb - 1 + j];
            const uint32_t cc = row[c];
            const uint32_t l = c > 0 ? row[c - 1] : 0u;
            const uint32_t r = c + 1 < DW ? row[c + 1] : 0u;
            h[j] = __builtin_amdgcn_alignbyte(cc, l, 3) + cc + __builtin_amdgcn_alignbyte(r, cc, 1);
            if (j >= 1 && j <= RL) C[j - 1] = cc;
        }
#pragma unroll
        for (int i = 0; i < RL; ++i) S[i] = h[i] + h[i + 1] + h[i + 2];
    };
    // Step z reads plane z+1 and writes the new plane z-1 (computed at the
    // previous step), so threads up to one step apart never touch a plane
    // that another reads or writes: one barrier per two steps suffices.
    for (int g = 1; g <= gens; ++g) {
        const int z_lo = g, z_hi = W - 1 - g;     // planes updated by this generation
        uint32_t Sp[RL], Sc[RL], Cc[RL], Cp[RL], pend[RL];
        if (worker) {
            plane_sums(z_lo - 1, Sp, Cp);
            plane_sums(z_lo, Sc, Cc);
        }
        __syncthreads();   // plane z_lo is read here and rewritten at step z_lo + 1
        for (int z = z_lo; z <= z_hi; ++z) {
            if (worker) {
                uint32_t Sn[RL], Cn[RL];
                plane_sums(z + 1, Sn, Cn);
#pragma unroll
                for (int i = 0; i < RL; ++i) {
                    if (z > z_lo) buf[z - 1][yb + i][c] = pend[i];
                    uint32_t res = rule_b6s567(Sp[i] + Sc[i] + Sn[i], Cc[i]);
                    if (!interior) res &= ca3k_keep_mask(gx, ys + yb + i, zs + z, n);
                    pend[i] = res;
                    Sp[i] = Sc[i];
                    Sc[i] = Sn[i];
                    Cc[i] = Cn[i];
                }
            }
            if ((z - z_lo) & 1) __syncthreads();
        }
        if ((z_hi - z_lo) % 2 == 0) __syncthreads();   // (uniform) the last step's reads are done
        if (worker) {
#pragma unroll
            for (int i = 0; i < RL; ++i) buf[z_hi][yb + i][c] = pend[i];
        }
        __syncthreads();
    }

    // 3. Write the tile: 8 dwords (32 cells) per tile row when RHO = 32.
    constexpr int TD = RHO / 4;                   // dwords per tile row
    for (int q = tid; q < RHO * RHO * TD; q += NT) {
        const int k = q % TD, yy = (q / TD) % RHO, zz = q / (TD * RHO);
        const int32_t gy = y0 + yy, gz = z0 + zz, x = x0 + 4 * k;
        if (gy + gz > n || x > n - gy - gz) continue;
        st_masked(out + (int64_t)gz * p2 + (int64_t)gy * p1, x, gy + gz, n, buf[KH + zz][KH + yy][KH / 4 + k]);
    }
}

// (the launch bound is Ca3kShape<RHO, KH, RL>::NT, written without commas)
template <int RHO, int KH, int RL, bool BB>
__global__ __launch_bounds__((((RHO + 2 * KH) / 4 * ((RHO + 2 * KH - 2) / RL) + 63) / 64) * 64) void k_ca3k(
    const Plan P, const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int gens)
{
    static_assert((((RHO + 2 * KH) / 4 * ((RHO + 2 * KH - 2) / RL) + 63) / 64) * 64 == Ca3kShape<RHO, KH, RL>::NT,
                  "launch bound");
    int32_t t[4] = {0, 0, 0, 0};
    const WgId g = wg_id(P);
    if (BB) {
        decode_bb(P, g.x, g.y, g.z, t);
    } else {
        if (!decode_h<3>(P, g.x, t)) return;
    }
    ca3k_tile<RHO, KH, RL>(P, in, out, t, gens);
}

}  // namespace smap
