// smap_plan.hpp -- host planner: (m, n, r, beta, rho, H|BB) -> Plan.
//
// Computes the side K of the block simplex, the native power-of-two part
// and the shell layers of the H launch (see smap_decode.hpp), the piece
// table of the fused launch and the workgroup counts.  Pure host integer
// code; no HIP calls.
#pragma once

#include <stdint.h>

#include "smap_decode.hpp"

namespace smap {

enum Status { kOk = 0, kEinval = -1, kEunsupported = -2, kErange = -3, kEhip = -4 };

struct PlanCounts {
    uint64_t launched = 0;
    uint64_t native = 0;
    uint64_t useful_tiles = 0;
    uint64_t full_tiles = 0;
};

// C(a, b) in 64 bits; returns false on overflow.
inline bool binom_u64(uint64_t a, uint64_t b, uint64_t *out)
{
    if (b > a) { *out = 0; return true; }
    if (b > a - b) b = a - b;
    unsigned __int128 r = 1;
    for (uint64_t i = 1; i <= b; ++i) {
        r = r * (a - b + i) / i;  // exact at every step
        if (r > (unsigned __int128)UINT64_MAX) return false;
    }
    *out = (uint64_t)r;
    return true;
}

inline uint64_t ipow_u64(uint64_t b, int e)
{
    uint64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// Workgroups of the native d-dim map of T_d(N-1), N = 2^j (levels: the
// level-ordered 3-D layout, sum over levels of 2^l c_l^3 = C(N+1, 3)).
inline uint64_t native_count(int d, int j, int beta, bool levels3 = false)
{
    if (d == 2) return h2_count(j);
    if (d == 3 && levels3) {
        uint64_t s = 0;
        for (int l = 0; l < j; ++l) s += (uint64_t(1) << l) * ipow_u64(uint64_t(1) << (j - 1 - l), 3);
        return s;
    }
    if (d == 3) return h3_count(j);
    uint64_t s = 0;  // d == 4: sum over levels of beta^l c_l^4
    for (int l = 0; l < j; ++l) s += ipow_u64((uint64_t)beta, l) * ipow_u64(uint64_t(1) << (j - 1 - l), 4);
    return s;
}

// Largest workgroup count any launch may use: the 1-D H grid is limited by
// the 32-bit work-item count of HIP's x dimension.
constexpr uint64_t kMaxWorkgroups = (uint64_t(1) << 31) / 256;

inline int make_plan(int m, int64_t n, int beta, int rho, bool bb, Plan *P, PlanCounts *C, int layout3 = 0)
{
    if (m < 2 || m > 4 || n < 0 || rho < 1) return kEinval;
    if (n > (int64_t)0x3FFFFFFF) return kErange;
    *P = Plan{};
    P->m = m;
    P->n = (int32_t)n;
    P->rho = rho;
    const int64_t M = n / rho;
    P->K = (int32_t)(M + 1);
    int64_t s = 1;
    for (int k = 0; k < m; ++k) {
        P->stride[k] = s;
        if ((unsigned __int128)s * (uint64_t)(n + 1) > ((unsigned __int128)1 << 56)) return kErange;
        s *= (n + 1);
    }
    PlanCounts cnt;
    if (!binom_u64((uint64_t)M + m, (uint64_t)m, &cnt.useful_tiles)) return kErange;
    // tiles lying entirely inside: sum(b) rho + m (rho - 1) <= n
    {
        const int64_t slack = n - (int64_t)m * (rho - 1);
        if (slack >= 0) {
            if (!binom_u64((uint64_t)(slack / rho) + m, (uint64_t)m, &cnt.full_tiles)) return kErange;
        }
    }
    if (bb) {
        const int64_t kb = (n + 1 + rho - 1) / rho;
        P->kbox = (int32_t)kb;
        P->kbox_div = make_divu((uint32_t)kb);
        // hardware grid limits: y and z (z = kbox^2 for m = 4) below 65536
        if (kb > 65535 || (m == 4 && kb * kb > 65535)) return kErange;
        uint64_t tot = 1;
        for (int k = 0; k < m; ++k) tot *= (uint64_t)kb;
        if (tot > UINT32_MAX) return kErange;
        P->total = (uint32_t)tot;
        cnt.launched = tot;
    } else {
        int j = (int)ilog2u((uint32_t)(M + 2));   // largest j with 2^j - 1 <= K
        P->j = j;
        P->L = (int32_t)(P->K - ((1 << j) - 1));
        P->beta = (m == 4) ? beta : 2;
        if (m == 4 && j > 8) return kErange;     // 4*lc shift width and count limits
        if (m == 3 && layout3) {
            if (j > 10) return kErange;          // 3*lc shift width
            P->layout3 = 1;
            P->nlvl = j;
            uint64_t acc = 0;
            for (int l = 0; l < j; ++l) {
                P->lvl_start[l] = (uint32_t)acc;
                acc += (uint64_t(1) << l) * ipow_u64(uint64_t(1) << (j - 1 - l), 3);
            }
            P->lvl_start[j] = (uint32_t)acc;
        }
        if (m == 4) {
            P->nlvl = j;
            uint64_t acc = 0;
            for (int l = 0; l < j; ++l) {
                P->lvl_start[l] = (uint32_t)acc;
                acc += ipow_u64((uint64_t)beta, l) * ipow_u64(uint64_t(1) << (j - 1 - l), 4);
            }
            P->lvl_start[j] = (uint32_t)acc;
        }
        uint64_t acc = native_count(m, j, beta, m == 3 && layout3);
        cnt.native = acc;
        P->piece_start[0] = 0;
        P->base_count[0] = (uint32_t)acc;
        P->npieces = 1;
        if (P->L > 0) {
            P->npieces = m;
            for (int p = 1; p < m; ++p) {
                const int d = m - p;
                const uint64_t base = (d == 1) ? (uint64_t)P->K : native_count(d, j, beta);
                P->piece_start[p] = (uint32_t)acc;
                P->base_count[p] = (uint32_t)base;
                acc += base * ipow_u64((uint64_t)P->L, m - d);
                if (acc > kMaxWorkgroups) return kErange;
            }
        }
        if (acc > kMaxWorkgroups) return kErange;
        P->piece_start[P->npieces] = (uint32_t)acc;
        P->total = (uint32_t)acc;
        for (int p = 0; p < P->npieces; ++p) P->base_div[p] = make_divu(P->base_count[p] ? P->base_count[p] : 1u);
        P->L_div = make_divu(P->L > 0 ? (uint32_t)P->L : 1u);
        cnt.launched = acc;
    }
    if (C) *C = cnt;
    return kOk;
}

}  // namespace smap
