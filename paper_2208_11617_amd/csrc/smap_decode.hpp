// smap_decode.hpp -- block-space maps: workgroup id -> tile of the block simplex.
//
// The box is cut into tiles of rho^m elements; the tiles meeting the simplex
// form the block simplex T_m(K) = { b in Z_+^m : b_1 + ... + b_m <= K-1 },
// K = floor(n/rho) + 1.  Each function here turns one workgroup id into the
// coordinates of one tile (or reports that the workgroup has no tile).  All
// of them are workgroup-uniform integer code (shifts, clz, adds), so on the
// GPU they live in scalar registers; the host build of the same code backs
// simplex_plan_tiles, so the decode the kernels run is also testable without
// a GPU.
//
// Coordinates here are 0-based: t[0] is b_1 (the x_1 tile index), etc.
//
// H, native part (N = 2^j).  The self-similar set S_N covers T_m(N-1), i.e.
// the tiles with sum <= N-2, as a cube of side N/2 plus beta recursive
// corner copies (Section 4.1, Lemma 1; Section 4.3, Lemma 3; Section 6,
// eq_generic-m with r = 1/2):
//   m = 2: Theorem 1 / eq_map2d on the grid Pi_{N/2, N-1}: b = 2^floor(log2(w_y+1)),
//          q = floor(w_x / b), (X, Y) = (w_x + q b, w_y + 2 q b + 1); the image
//          is { 0 <= X < Y <= N-1 } and becomes the tile (X, N-1-Y).
//   m = 3: the packed grid (N/2) x (N/2) x (N/2 + N/4) of Section 4.3: the
//          first cube takes w_z < N/2; above it the 2-D (b, q) decode of
//          eq_map2d places the cubes of the smaller levels, the stack slot
//          being w_z - N/2 < b.  A cube cell whose local coordinates sum to
//          2b-1 or more lies outside the simplex and is reflected by the
//          hinge (b-1-l_1, b-1-l_2, 2b-1-l_3) onto the third corner of its
//          sub-simplex, which it covers exactly (the printed hinge has the
//          z-term 2b-1-L_z; the reflection that lands in the simplex is the
//          local z' = 2b-1-l_z, i.e. a shift of 2b-1-2 l_z).
//   m = 4: levels l = 0..j-1 laid out one after another, level l holding
//          beta^l cubes of side c = N/2^(l+1); the copy index is read in base
//          beta, digit k choosing the corner axis at recursion depth k.
//          beta = 3: the fourth corner is reached by the same hinge
//          (c-1-l_1, c-1-l_2, c-1-l_3, 2c-1-l_4) -- exact for cells whose local
//          sum is >= 3c-2; cells with 2c-1 <= sum <= 3c-3 are discarded.
//          beta = 4: no hinge; every cube cell with sum >= 2c-1 is discarded.
//          The launched count equals eq_generic-m with r = 1/2:
//          (N^4 - beta^j) / (16 - beta).
//
// H, general K.  With N = 2^j the largest power of two such that N-1 <= K,
// T_m(K) = T_m(N-1) plus L = K-(N-1) shell layers (sum in [N-1, K-1]).  Every
// shell tile b is reached from its prefix sums S_d = b_1 + ... + b_d: for the
// first d with S_{d+1} >= N-1 the tile is (base, layers) with base
// (b_1..b_d) in T_d(N-1) (d >= 2, decoded by the native d-dim map) or
// b_1 in [0, K) (d = 1), and layer indices i_k = S_{k+1} - (N-1) in [0, L) for
// k = d..m-1.  Piece d launches base x L^(m-d) workgroups; the ones whose
// layer indices decrease, or (d = 1) whose b_2 would be negative, are
// discarded.  This plays the role of Section 4.2's trapezoids (a native
// triangle plus rectangular pieces, fused into one launch).
//
// BB (Section 2): the tile is the workgroup's grid coordinate, f(x) = x; m = 4
// is linearised into a 3-D grid (z = b_3 + kbox * b_4).
#pragma once

#include <stdint.h>

#ifndef SMAP_HD
#if defined(__HIPCC__)
#define SMAP_HD __host__ __device__ __forceinline__
#else
#define SMAP_HD inline
#endif
#endif

namespace smap {

constexpr int kMaxLevels = 16;

// Division by a workgroup-uniform divisor d >= 1 through a multiplier
// computed once on the host (Granlund and Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994, the unsigned
// round-up method for 32-bit words): exact for every 32-bit x.  On the GPU
// it is a scalar multiply-high, a subtract, an add and two shifts.
struct Divu {
    uint32_t d, m, sh1, sh2;
};

SMAP_HD Divu make_divu(uint32_t d)
{
    uint32_t l = 0;  // ceil(log2 d)
    while ((uint64_t(1) << l) < (uint64_t)d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1u;
    return Divu{d, (uint32_t)m, l < 1u ? l : 1u, l > 1u ? l - 1u : 0u};
}

SMAP_HD uint32_t divu(uint32_t x, uint32_t m, uint32_t sh1, uint32_t sh2)
{
    const uint32_t t1 = (uint32_t)(((uint64_t)m * x) >> 32);
    return (t1 + ((x - t1) >> sh1)) >> sh2;
}

SMAP_HD uint32_t divu(uint32_t x, const Divu &D) { return divu(x, D.m, D.sh1, D.sh2); }

// Everything a kernel needs to decode its workgroup id.  Passed by value in
// the kernel arguments (it ends up in scalar registers / the constant cache).
struct Plan {
    int32_t m;
    int32_t n;
    int32_t rho;
    int32_t K;          // side of the block simplex
    int32_t j;          // native N = 2^j (H only)
    int32_t L;          // shell layers (H only)
    int32_t beta;       // replication for the 4-D native map (3 or 4)
    int32_t kbox;       // tiles per axis of the BB launch
    int32_t npieces;    // 1 (native only) or m (native + m-1 shell pieces)
    int32_t nlvl;       // levels of the 4-D native map
    uint32_t total;     // launched workgroups
    uint32_t piece_start[5];     // piece p = 0 (native), 1..m-1 (shell d = m-p)
    uint32_t base_count[4];      // workgroups of the base map of each piece
    uint32_t lvl_start[kMaxLevels + 1];
    int64_t stride[4];           // element strides (n+1)^k
    Divu base_div[4];            // division by base_count[p]
    Divu L_div;                  // division by L (1 when there is no shell)
    Divu kbox_div;               // division by kbox (BB, m = 4)
    uint32_t grid[3];            // launch grid of this launch (set per launch)
    Divu grid_div[2];            // division by grid[0], grid[1] (set per launch)
    uint32_t nwg;                // grid[0] * grid[1] * grid[2] (< 2^32)
    uint32_t remap;              // workgroup order: 0 hardware, 1 xcd_remap, 2 xcd_scatter
    int32_t layout3;             // m = 3 native part: 0 packed grid, 1 one range per level
    uint32_t wg_base;            // first map index of this launch (0; a piece's start when
                                 // the pieces run as launches of their own)
};

// Launch order.  The 8 XCDs of the chip each have their own L2; workgroup L
// (x fastest, then y, then z) is dispatched to XCD L mod 8.  Renumbering
// L -> xcd_remap(L) gives each XCD one contiguous range of logical ids, so
// neighbouring tiles (which share cache lines at their row ends and halo
// rows) run on the same XCD at about the same time.  A bijection of
// [0, nwg): XCD x holds the cnt(x) = nwg/8 + (x < nwg mod 8) ids starting at
// x * (nwg/8) + min(x, nwg mod 8).
SMAP_HD uint32_t xcd_remap(uint32_t L, uint32_t nwg)
{
    const uint32_t per = nwg >> 3, rem = nwg & 7u;
    const uint32_t x = L & 7u;
    return x * per + (x < rem ? x : rem) + (L >> 3);
}

// BB launches: L -> xcd_scatter(L) rotates the ids inside each aligned group
// of 8 by a pseudo-random amount (the top three bits of a multiplicative
// hash of the group index), so the workgroups of one grid column meet every
// XCD.  In the plain order an x extent that shares a factor with 8 ties each
// column of box tiles to fixed XCDs, and the simplex's work sits in the low
// columns: with 4 tiles per side the 3-D step ran 2.5x longer than with 3
// or 5.  Ids stay inside their group, so the order is otherwise unchanged;
// a last, partial group keeps its ids.  A bijection of [0, nwg).
SMAP_HD uint32_t xcd_scatter(uint32_t L, uint32_t nwg)
{
    if ((L | 7u) >= nwg) return L;
    const uint32_t h = ((L >> 3) * 0x9E3779B1u) >> 29;
    return (L & ~7u) | ((L + h) & 7u);
}

#if defined(__HIPCC__)
// Logical workgroup coordinates of this workgroup in the launch grid.
struct WgId {
    uint32_t x, y, z;
};
__device__ __forceinline__ WgId wg_id(const Plan &P)
{
    if (P.remap) {
        if (P.remap == 1 && P.grid[1] == 1 && P.grid[2] == 1)
            return {xcd_remap(blockIdx.x, P.nwg), 0u, 0u};  // 1-D: no division
        const uint32_t L = (blockIdx.z * P.grid[1] + blockIdx.y) * P.grid[0] + blockIdx.x;
        const uint32_t g = P.remap == 1 ? xcd_remap(L, P.nwg) : xcd_scatter(L, P.nwg);
        const uint32_t r = divu(g, P.grid_div[0]), r2 = divu(r, P.grid_div[1]);
        return {g - r * P.grid[0], r - r2 * P.grid[1], r2};
    }
    return {blockIdx.x, blockIdx.y, blockIdx.z};
}
#endif

#if defined(__HIPCC__)
// Workgroup barrier that orders LDS only: waits for this wave's LDS
// operations, then s_barrier, with fences restricted to the local address
// space.  __syncthreads() also waits for every outstanding global load and
// store (a workgroup-scope fence covers global memory), which would drain the
// loads that the tile walks keep in flight across barriers; no kernel here
// passes global-memory data between the waves of a workgroup.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
#endif

SMAP_HD uint32_t ilog2u(uint32_t v)  // floor(log2 v), v > 0: 31 - clz(v)
{
    return 31u - (uint32_t)__builtin_clz(v);
}

// ---- native counts -------------------------------------------------------

SMAP_HD uint64_t h2_count(int j) { return (uint64_t(1) << (j - 1)) * ((uint64_t(1) << j) - 1); }

SMAP_HD uint64_t h3_count(int j)
{
    uint64_t c0 = uint64_t(1) << (j - 1);
    return c0 * c0 * (c0 + (c0 >> 1));
}

// ---- native decodes ------------------------------------------------------

// Theorem 1 / eq_map2d.  Always lands on a tile of T_2(N-1).
SMAP_HD void h2_native(int j, uint32_t w, int32_t *t)
{
    const uint32_t lh = (uint32_t)j - 1u;
    const uint32_t wx = w & ((1u << lh) - 1u);
    const uint32_t wy = w >> lh;
    const uint32_t lb = ilog2u(wy + 1u);          // b = 2^lb
    const uint32_t q = wx >> lb;                  // q = floor(w_x / b)
    const uint32_t X = wx + (q << lb);            // w_x + q b
    const uint32_t Y = wy + (q << (lb + 1u)) + 1u; // w_y + 2 q b + 1
    t[0] = (int32_t)X;
    t[1] = (int32_t)((1u << j) - 1u - Y);
}

// Packed 3-D grid with the hinge.  Returns false for the unused slots.
SMAP_HD bool h3_native(int j, uint32_t w, int32_t *t)
{
    const uint32_t lc0 = (uint32_t)j - 1u;
    const uint32_t c0 = 1u << lc0;
    const uint32_t wx = w & (c0 - 1u);
    const uint32_t wy = (w >> lc0) & (c0 - 1u);
    const uint32_t wz = w >> (2u * lc0);
    int32_t o0, o1, cb, l0, l1, l2;
    if (wz < c0) {  // the first cube, at the origin
        o0 = 0; o1 = 0; cb = (int32_t)c0;
        l0 = (int32_t)wx; l1 = (int32_t)wy; l2 = (int32_t)wz;
    } else {
        const uint32_t lb = ilog2u(wy + 1u);
        if (lb >= lc0) return false;              // last row: no level of side N/2 here
        const uint32_t bb = 1u << lb;
        const uint32_t z = wz - c0;
        if (z >= bb) return false;                // stack slot above a smaller cube
        const uint32_t q = wx >> lb;
        cb = (int32_t)bb;
        l0 = (int32_t)(wx & (bb - 1u));
        l1 = (int32_t)(bb - 1u - (wy + 1u - bb));
        l2 = (int32_t)z;
        o0 = (int32_t)(q << (lb + 1u));
        o1 = (int32_t)((1u << j) - (bb << 1) - (q << (lb + 1u)));
    }
    if (l0 + l1 + l2 >= 2 * cb - 1) {             // hinge onto the third corner
        t[0] = o0 + cb - 1 - l0;
        t[1] = o1 + cb - 1 - l1;
        t[2] = 2 * cb - 1 - l2;
    } else {
        t[0] = o0 + l0;
        t[1] = o1 + l1;
        t[2] = l2;
    }
    return true;
}

// Level-ordered 3-D map (the fully efficient variant: one range of
// workgroups per level, here concatenated into one launch).  Level l holds
// 2^l cubes of side c = N/2^(l+1); the copy index is read in base 2, digit k
// choosing the corner axis (x_1 or x_2) at recursion depth k, and the cube
// cells whose local sum is 2c-1 or more are reflected by the hinge onto the
// x_3 corner, which they cover exactly: every workgroup lands on a tile.
// The level and the corner offsets have closed forms (no per-level scan).
SMAP_HD bool h3_levels(const Plan &P, uint32_t w, int32_t *t)
{
    // Level l starts at (N^3 - N^3/4^l) / 6 (the sizes N^3/8 4^-l form a
    // geometric series), so with D = N^3 - 6w the level is the largest l
    // with D <= 2^(3j - 2l): l = floor((3j - ceil(log2 D)) / 2), one count of
    // leading zeros.  N^3 <= 2^30 (the planner caps j at 10).
    const uint32_t j = (uint32_t)P.j;
    const uint32_t N3 = 1u << (3u * j);
    const uint32_t D = N3 - 6u * w;              // > N >= 2 for every launched w
    const uint32_t cl = 32u - (uint32_t)__builtin_clz(D - 1u);   // ceil(log2 D)
    const uint32_t l = (3u * j - cl) >> 1;
    const uint32_t start = (N3 - (1u << (3u * j - 2u * l))) / 6u;
    const uint32_t i = w - start;
    const uint32_t lc = j - 1u - l;
    const uint32_t c = 1u << lc;
    const uint32_t l0 = i & (c - 1u), l1 = (i >> lc) & (c - 1u), l2 = (i >> (2u * lc)) & (c - 1u);
    // copy q (l binary digits): digit 1 at depth k shifts by N/2^k along x_2,
    // digit 0 along x_1, so the x_2 offset is q N/2^l and the two offsets
    // add up to N - N/2^l
    const uint32_t q = i >> (3u * lc);
    const int32_t o1 = (int32_t)(q << (j - l));
    const int32_t o0 = (int32_t)((1u << j) - ((1u << j) >> l)) - o1;
    const int32_t ci = (int32_t)c;
    if ((int32_t)(l0 + l1 + l2) >= 2 * ci - 1) {   // hinge onto the x_3 corner
        t[0] = o0 + ci - 1 - (int32_t)l0;
        t[1] = o1 + ci - 1 - (int32_t)l1;
        t[2] = 2 * ci - 1 - (int32_t)l2;
    } else {
        t[0] = o0 + (int32_t)l0;
        t[1] = o1 + (int32_t)l1;
        t[2] = (int32_t)l2;
    }
    return true;
}

// Level-ordered 4-D map with replication beta (3: hinge, 4: none).
SMAP_HD bool h4_native(const Plan &P, uint32_t w, int32_t *t)
{
    // level: last l with lvl_start[l] <= w (unrolled: no runtime-indexed reads)
    int l = 0;
    uint32_t start = 0;
#pragma unroll
    for (int k = 1; k < kMaxLevels; ++k) {
        if (k < P.nlvl && w >= P.lvl_start[k]) {
            l = k;
            start = P.lvl_start[k];
        }
    }
    const uint32_t i = w - start;
    const uint32_t lc = (uint32_t)(P.j - 1 - l);
    const uint32_t c = 1u << lc;
    const uint32_t cell = i & ((1u << (4u * lc)) - 1u);
    uint32_t q = i >> (4u * lc);
    int32_t lam[4], o[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) lam[k] = (int32_t)((cell >> (uint32_t(k) * lc)) & (c - 1u));
    const bool b4 = P.beta == 4;                  // beta is 3 or 4: constant divisors
    for (int k = l; k >= 1; --k) {                // corner chosen at depth k
        const uint32_t q3 = q / 3u;
        const uint32_t d = b4 ? (q & 3u) : q - 3u * q3;
        q = b4 ? (q >> 2) : q3;
        const int32_t step = (int32_t)((1u << P.j) >> k);
        // select the axis without a dynamically indexed array (no scratch)
        o[0] += d == 0u ? step : 0;
        o[1] += d == 1u ? step : 0;
        o[2] += d == 2u ? step : 0;
        o[3] += d == 3u ? step : 0;
    }
    const int32_t ci = (int32_t)c;
    const int32_t s = lam[0] + lam[1] + lam[2] + lam[3];
    if (s >= 2 * ci - 1) {
        if (P.beta == 4 || s < 3 * ci - 2) return false;
        t[0] = o[0] + ci - 1 - lam[0];
        t[1] = o[1] + ci - 1 - lam[1];
        t[2] = o[2] + ci - 1 - lam[2];
        t[3] = o[3] + 2 * ci - 1 - lam[3];
    } else {
        for (int k = 0; k < 4; ++k) t[k] = o[k] + lam[k];
    }
    return true;
}

// ---- H: native + shell pieces ------------------------------------------------

template <int M>
SMAP_HD bool decode_h(const Plan &P, uint32_t w, int32_t *t)
{
    constexpr int m = M;
    w += P.wg_base;
    // piece: last p with piece_start[p] <= w (unrolled: no runtime-indexed reads)
    // (scalar fields selected one by one: a selected struct or array element
    // would be turned into a runtime-indexed local copy in scratch memory)
    int p = 0;
    uint32_t pstart = 0, bc = P.base_count[0];
    uint32_t bm = P.base_div[0].m, bs1 = P.base_div[0].sh1, bs2 = P.base_div[0].sh2;
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const bool in_k = k < P.npieces && w >= P.piece_start[k];
        p = in_k ? k : p;
        pstart = in_k ? P.piece_start[k] : pstart;
        bc = in_k ? P.base_count[k] : bc;
        bm = in_k ? P.base_div[k].m : bm;
        bs1 = in_k ? P.base_div[k].sh1 : bs1;
        bs2 = in_k ? P.base_div[k].sh2 : bs2;
    }
    const uint32_t loc = w - pstart;
    if (p == 0) {
        if constexpr (M == 2) { h2_native(P.j, loc, t); return true; }
        else if constexpr (M == 3) return P.layout3 ? h3_levels(P, loc, t) : h3_native(P.j, loc, t);
        else return h4_native(P, loc, t);
    }
    const int d = m - p;                          // base dimension of this piece
    uint32_t lay = divu(loc, bm, bs1, bs2);
    const uint32_t base = loc - lay * bc;
    if (d == 1) {
        t[0] = (int32_t)base;
    } else if (d == 2) {
        h2_native(P.j, base, t);
    } else if constexpr (M == 4) {
        if (!h3_native(P.j, base, t)) return false;
    }
    const int32_t h = (1 << P.j) - 1;
    const uint32_t L = (uint32_t)P.L;
    // Compile-time indices only (the coordinates stay in registers).
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < d) s += t[k];
    bool ok = true;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        if (k >= d && k < m) {
            const uint32_t next = divu(lay, P.L_div);
            const int32_t ik = (int32_t)(lay - next * L);
            lay = next;
            t[k] = h + ik - s;
            ok = ok && t[k] >= 0;
            s = h + ik;
        }
    }
    return ok;
}

SMAP_HD bool decode_h_rt(const Plan &P, uint32_t w, int32_t *t)  // host-side dispatch on m
{
    if (P.m == 2) return decode_h<2>(P, w, t);
    if (P.m == 3) return decode_h<3>(P, w, t);
    return decode_h<4>(P, w, t);
}

// ---- BB ---------------------------------------------------------------------

SMAP_HD void decode_bb(const Plan &P, uint32_t gx, uint32_t gy, uint32_t gz, int32_t *t)
{
    t[0] = (int32_t)gx;
    t[1] = (int32_t)gy;
    if (P.m == 3) t[2] = (int32_t)gz;
    if (P.m == 4) {
        const uint32_t q = divu(gz, P.kbox_div);
        t[2] = (int32_t)(gz - q * (uint32_t)P.kbox);
        t[3] = (int32_t)q;
    }
}

}  // namespace smap
