// smap_lib.hip -- the C ABI declared in include/simplexmap.h.
//
// Validates arguments, looks up (or builds) the launch plan, and enqueues
// the kernel for (op, m, rho, H|BB) on the caller's stream.  The only state
// is the per-process tile table (simplex_set_tile) and the plan cache, both
// behind one mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/simplexmap.h"
#include "smap_batch.hpp"
#include "smap_ca2.hpp"
#include "smap_ca2k.hpp"
#include "smap_ca3k.hpp"
#include "smap_ca3.hpp"
#include "smap_copy.hpp"
#include "smap_plan.hpp"
#include "smap_point.hpp"
#include "smap_serve.hpp"

using namespace smap;

namespace {

struct TileCfg {
    int rho;
    int wg;
    int sub;      // workgroups per tile (CA2 splits a tile into row sub-blocks)
    int grp = 1;  // tiles per workgroup (pointwise ops: x_1-adjacent map units)
};

// CA2 shapes: (rho, threads) -> waves W, rows per wave R, sub-blocks per tile.
struct Ca2Shape {
    int rho, wg, w, r, sub;
};
constexpr Ca2Shape kCa2Shapes[] = {
    {1024, 64, 1, 4, 256}, {1024, 128, 2, 16, 32}, {1024, 256, 4, 16, 16},
    {512, 512, 8, 16, 2},  {256, 256, 4, 16, 1},   {128, 128, 2, 8, 1},
    // waves side by side along x: 1 KB columns, 2 or 4 per workgroup
    {2048, 128, 2, 16, 128}, {2048, 256, 4, 16, 64}, {4096, 256, 4, 16, 256},
};

// Pointwise shapes: (m, rho) -> threads, sub-blocks per tile, tiles per
// workgroup.  The first listed shape of an m is its default; the first
// listed grouping of an (m, rho, threads) is the one simplex_set_tile picks.
struct PointShape {
    int m, rho, wg, sub, grp;
};
constexpr PointShape kPointShapes[] = {
    {2, 32, 256, 1, 1}, {2, 16, 64, 1, 1}, {2, 64, 256, 1, 1}, {2, 128, 256, 2, 1},
    {3, 16, 256, 1, 1}, {3, 8, 128, 1, 1}, {3, 32, 256, 4, 1},
    // m = 4: two x_1-adjacent rho = 8 tiles per workgroup (64-byte row runs)
    {4, 8, 256, 1, 2},  {4, 4, 64, 1, 1},  {4, 16, 256, 16, 1},
    // several x_1-adjacent tiles per workgroup, or one
    {4, 8, 256, 1, 1},  {4, 8, 256, 1, 4}, {4, 8, 128, 1, 4}, {4, 8, 256, 1, 8},
    {4, 4, 256, 1, 8},  {4, 4, 256, 1, 16},
    {3, 16, 256, 1, 2}, {3, 8, 256, 1, 4},
    // one wave per workgroup: the scalar decode runs once per workgroup
    {4, 8, 64, 1, 1},   {4, 8, 64, 1, 2},  {4, 8, 64, 1, 4},  {4, 8, 128, 1, 2},
    {3, 16, 64, 1, 1},  {3, 16, 64, 1, 2}, {2, 32, 64, 1, 1}, {2, 32, 64, 1, 2},
};

// CA3 shapes: (rho, threads) -> rows RY (y), planes RZ (z), rows per lane RL.
// Sub-blocks are 8 planes deep (4 and 16 measured slower at rho = 256).
struct Ca3Shape {
    int rho, wg, ry, rz, rl, sub;
};
constexpr int kCa3Rz = 8;
constexpr int ca3_rz(int rho) { return kCa3Rz < rho ? kCa3Rz : rho; }
constexpr Ca3Shape kCa3Shapes[] = {
    {128, 256, 32, ca3_rz(128), 1, (128 / 32) * (128 / ca3_rz(128))},
    {128, 128, 16, ca3_rz(128), 1, (128 / 16) * (128 / ca3_rz(128))},
    {128, 512, 64, ca3_rz(128), 1, (128 / 64) * (128 / ca3_rz(128))},
    {256, 256, 16, ca3_rz(256), 1, (256 / 16) * (256 / ca3_rz(256))},
    {256, 128, 8, ca3_rz(256), 1, (256 / 8) * (256 / ca3_rz(256))},
    {256, 512, 32, ca3_rz(256), 1, (256 / 32) * (256 / ca3_rz(256))},
    {64, 128, 64, ca3_rz(64), 2, (64 / 64) * (64 / ca3_rz(64))},
    {64, 256, 64, ca3_rz(64), 1, (64 / 64) * (64 / ca3_rz(64))},
    {32, 64, 32, ca3_rz(32), 1, (32 / 32) * (32 / ca3_rz(32))},
};

// op class: 0 = pointwise (MAP/ACCUM/HITS/HASH), 1 = CA2, 2 = CA3
int op_class(int op) { return op == OP_CA2 ? 1 : (op == OP_CA3 ? 2 : 0); }

// CA3: 256^3 tiles from n = 768 on; below, 128^3 (with only two or three
// 256-cell tiles per side most of their sub-blocks fall outside the simplex)
constexpr int64_t kCa3LargeTileN = 768;

TileCfg default_tile(int m, int64_t n, int cls)
{
    if (cls == 1) return {1024, 64, 256};
    if (cls == 2) {  // the first listed shape of the tile side (256 threads)
        const int rho = n >= kCa3LargeTileN ? 256 : 128;
        for (const Ca3Shape &c : kCa3Shapes)
            if (c.rho == rho) return {c.rho, c.wg, c.sub};
    }
    for (const PointShape &c : kPointShapes)  // the first listed shape of an m is its default
        if (c.m == m) return {c.rho, c.wg, c.sub, c.grp};
    return {0, 0, 1};
}

// The compiled shape of (m, class, rho, threads, tiles per workgroup);
// *wg = 0 or *grp = 0 take the first listed match.  The automata have no
// grouping (*grp must be 0 or 1).
bool tile_supported(int m, int cls, int rho, int *wg, int *sub, int *grp)
{
    *sub = 1;
    if (cls == 0) {
        for (const PointShape &c : kPointShapes) {
            if (c.m == m && c.rho == rho && (*wg == 0 || *wg == c.wg) && (*grp == 0 || *grp == c.grp)) {
                *wg = c.wg;
                *sub = c.sub;
                *grp = c.grp;
                return true;
            }
        }
        return false;
    }
    if (*grp > 1) return false;
    *grp = 1;
    if (cls == 1) {  // the first listed shape of a rho is its default
        for (const Ca2Shape &c : kCa2Shapes) {
            if (c.rho == rho && (*wg == 0 || *wg == c.wg)) {
                *wg = c.wg;
                *sub = c.sub;
                return true;
            }
        }
        return false;
    }
    if (m != 3) return false;
    for (const Ca3Shape &c : kCa3Shapes) {
        if (c.rho == rho && (*wg == 0 || *wg == c.wg)) {
            *wg = c.wg;
            *sub = c.sub;
            return true;
        }
    }
    return false;
}

std::mutex g_mu;
std::map<std::pair<int, int>, TileCfg> g_tiles;  // (m, class) -> override

struct CachedPlan {
    Plan plan;
    PlanCounts counts;
    int status;
};
std::map<std::tuple<int, int64_t, int, int, int, int, int>, CachedPlan> g_plans;  // (m,n,beta,rho,bb,cls,layout)
// H native layout for m = 3 (simplex_set_layout); SMAP_LAYOUT_AUTO: the
// level-ordered layout for one-job CA3 launches (one step or several
// generations) and their plans, the packed one for everything else
int g_layout3 = SMAP_LAYOUT_AUTO;
int g_general = 0;  // H launch of the pieces: 0 fused, 1 one launch per piece (simplex_set_general)

TileCfg tile_for(int m, int64_t n, int cls)
{
    auto it = g_tiles.find({m, cls});
    return it != g_tiles.end() ? it->second : default_tile(m, n, cls);
}

// Autotuned H choices per (m, n, op class) (g_mu held when used).
struct Tuned {
    TileCfg t;
    int beta;
};
std::map<std::tuple<int, int64_t, int>, Tuned> g_tuned;

TileCfg tile_for_h(int m, int64_t n, int cls)
{
    auto it = g_tuned.find(std::make_tuple(m, n, cls));
    return it != g_tuned.end() ? it->second.t : tile_for(m, n, cls);
}

int resolve_rb(int m, int r, int beta, int *beta_out)
{
    if (r != 0 && r != 2) return kEunsupported;
    if (beta == 0) beta = (m == 4) ? 3 : 2;
    if (m == 2 || m == 3) {
        if (beta != 2) return kEunsupported;
    } else if (beta != 3 && beta != 4) {
        return kEunsupported;
    }
    *beta_out = beta;
    return kOk;
}

bool box_elems(int m, int64_t n, int64_t *out)
{
    __int128 e = 1;
    for (int k = 0; k < m; ++k) {
        e *= (__int128)(n + 1);
        if (e > ((__int128)1 << 56)) return false;
    }
    *out = (int64_t)e;
    return true;
}

// Plan lookup; also checks that in-tile offsets fit the kernels' 32-bit
// lane offsets.
// Plan of (m, n, beta, tile t, H|BB, op class) from the cache (g_mu held).
int plan_for(int m, int64_t n, int beta, bool bb, int cls, const TileCfg &t, Plan *P, PlanCounts *C,
             bool one_job = false)
{
    int lay = 0;
    if (m == 3 && !bb)
        lay = g_layout3 != SMAP_LAYOUT_AUTO ? g_layout3
                                            : (one_job && cls == 2 ? SMAP_LAYOUT_LEVELS : SMAP_LAYOUT_PACKED);
    auto key = std::make_tuple(m, n, bb ? 0 : beta, t.rho, bb ? 1 : 0, cls, lay);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        CachedPlan cp{};
        cp.status = make_plan(m, n, beta, t.rho, bb, &cp.plan, &cp.counts, lay);
        if (cp.status == kOk && !bb && (uint64_t)cp.plan.total * (uint64_t)t.sub > kMaxWorkgroups)
            cp.status = kErange;
        if (cp.status == kOk && bb) {
            const uint64_t kb = (uint64_t)cp.plan.kbox;
            const uint64_t zext = (m == 2) ? (cls == 1 ? kb : 1) : (m == 3 ? kb : kb * kb);
            if (zext * (uint64_t)t.sub > 65535) cp.status = kErange;
            // workgroups are renumbered with 32-bit linear ids
            if ((uint64_t)cp.plan.total * (uint64_t)t.sub > UINT32_MAX) cp.status = kErange;
        }
        if (cp.status == kOk) {
            // The kernels use unsigned 32-bit offsets below a 64-bit base: the
            // pointwise kernels inside one tile (element index), the automata
            // inside one plane (CA3) or one sub-block of rows (CA2).
            __int128 span = 0;
            if (cls == 0) {
                for (int k = 0; k < m; ++k) span += (__int128)(t.rho + 1) * cp.plan.stride[k];
            } else {
                span = (__int128)cp.plan.stride[m - 1] * (t.rho + 2) + 64;
                if (cls == 2) span = (__int128)cp.plan.stride[2] + (__int128)cp.plan.stride[1] * 2 + 64;
            }
            if (span >= ((__int128)1 << 32)) cp.status = kErange;
        }
        if (g_plans.size() > 4096) g_plans.clear();
        it = g_plans.emplace(key, cp).first;
    }
    *P = it->second.plan;
    if (C) *C = it->second.counts;
    return it->second.status;
}

// Plan for a launch with the current tile of (m, op class).
int get_plan(int m, int64_t n, int beta, int op, bool bb, Plan *P, PlanCounts *C, TileCfg *tc)
{
    const int cls = op_class(op);
    std::lock_guard<std::mutex> lk(g_mu);
    const TileCfg t = bb ? tile_for(m, n, cls) : tile_for_h(m, n, cls);
    *tc = t;
    return plan_for(m, n, beta, bb, cls, t, P, C, true);
}

int check_op(int m, int64_t n, int op)
{
    if (m < 2 || m > 4 || n < 0) return kEinval;
    if (op < OP_MAP || op > OP_EDM) return kEinval;
    if ((op == OP_CA2 || op == OP_EDM) && m != 2) return kEinval;
    if (op == OP_CA3 && m != 3) return kEinval;
    return kOk;
}

int check_buffers(int m, int64_t n, int op, const void *in, const void *out)
{
    int64_t elems;
    if (!box_elems(m, n, &elems)) return kErange;
    if (op == OP_ACCUM && (!in || !out)) return kEinval;
    if ((op == OP_HITS || op == OP_HASH) && !out) return kEinval;
    if (op == OP_EDM && (!in || !out || ((uintptr_t)in & 15u) != 0)) return kEinval;  // 16-byte aligned points
    if (op == OP_CA2 || op == OP_CA3) {
        if (!in || !out) return kEinval;
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        const uintptr_t len = (uintptr_t)elems;
        if (a < b + len && b < a + len) return kEinval;  // overlapping ping-pong buffers
    }
    if (op == OP_ACCUM && in != out) {
        // in place (in == out) is allowed; any other overlap would race
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        const uintptr_t len = (uintptr_t)elems * 4u;
        if (a < b + len && b < a + len) return kEinval;
    }
    return kOk;
}

// The buffers of a batch: no job's output may overlap another job's output
// or input (inputs may be shared).  Each job's own pair is checked by
// check_buffers.  Sorts the output intervals, checks neighbours, then
// looks up each input among the outputs: O(k log k).
int check_batch_buffers(const simplex_job *jobs, int32_t njobs)
{
    struct Iv {
        uintptr_t a, b;
        int32_t job;
    };
    std::vector<Iv> outs;
    outs.reserve((size_t)njobs);
    for (int32_t i = 0; i < njobs; ++i) {
        int64_t elems = 0;
        if (!box_elems(jobs[i].m, jobs[i].n, &elems)) return kErange;
        const uintptr_t o = (uintptr_t)jobs[i].buf_out;
        outs.push_back({o, o + (uintptr_t)elems, i});
    }
    std::sort(outs.begin(), outs.end(), [](const Iv &x, const Iv &y) { return x.a < y.a; });
    for (size_t k = 1; k < outs.size(); ++k)
        if (outs[k].a < outs[k - 1].b) return kEinval;    // two outputs overlap
    // sorted, disjoint outputs have sorted ends: the last output that starts
    // before an input's end is the only one that can reach into it
    for (int32_t i = 0; i < njobs; ++i) {
        int64_t elems = 0;
        box_elems(jobs[i].m, jobs[i].n, &elems);
        const uintptr_t a = (uintptr_t)jobs[i].buf_in, b = a + (uintptr_t)elems;
        auto it = std::lower_bound(outs.begin(), outs.end(), b,
                                   [](const Iv &x, uintptr_t v) { return x.a < v; });
        if (it == outs.begin()) continue;
        --it;
        if (it->b > a && it->job != i) return kEinval;    // another job writes this input
    }
    return kOk;
}

template <int M, int RHO, int NT, int SUB, int OP, bool BB>
void launch_point(const Plan &P, dim3 grid, const void *in, void *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_point<M, RHO, NT, OP, BB, SUB>), grid, dim3(NT), 0, s, P,
                       (const uint32_t *)in, (uint32_t *)out);
}

template <int M, int RHO, int NT, int OP, bool BB, int U>
void launch_point_grp(const Plan &P, dim3 grid, const void *in, void *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_point_grp<M, RHO, NT, OP, BB, U>), grid, dim3(NT), 0, s, P,
                       (const uint32_t *)in, (uint32_t *)out);
}

template <int OP, bool BB>
int dispatch_point_shape(int m, const TileCfg &tc, const Plan &P, dim3 grid, const void *in, void *out,
                         hipStream_t s)
{
    const int64_t key = ((int64_t)m * 10000 + tc.rho) * 100000 + (int64_t)tc.wg * 100 + tc.grp;
    switch (key) {
#define SMAP_PT(M, RHO, NT, SUB) \
    case ((int64_t)M * 10000 + RHO) * 100000 + NT * 100 + 1: launch_point<M, RHO, NT, SUB, OP, BB>(P, grid, in, out, s); return kOk;
#define SMAP_PTG(M, RHO, NT, U) \
    case ((int64_t)M * 10000 + RHO) * 100000 + NT * 100 + U: launch_point_grp<M, RHO, NT, OP, BB, U>(P, grid, in, out, s); return kOk;
    SMAP_PT(2, 32, 256, 1)
    SMAP_PT(2, 16, 64, 1)
    SMAP_PT(2, 64, 256, 1)
    SMAP_PT(2, 128, 256, 2)
    SMAP_PT(3, 16, 256, 1)
    SMAP_PT(3, 8, 128, 1)
    SMAP_PT(3, 32, 256, 4)
    SMAP_PT(4, 8, 256, 1)
    SMAP_PT(4, 4, 64, 1)
    SMAP_PT(4, 16, 256, 16)
    SMAP_PT(4, 8, 64, 1)
    SMAP_PT(3, 16, 64, 1)
    SMAP_PT(2, 32, 64, 1)
    SMAP_PTG(4, 8, 64, 2)
    SMAP_PTG(4, 8, 64, 4)
    SMAP_PTG(4, 8, 128, 2)
    SMAP_PTG(3, 16, 64, 2)
    SMAP_PTG(2, 32, 64, 2)
    SMAP_PTG(4, 8, 256, 4)
    SMAP_PTG(4, 8, 128, 4)
    SMAP_PTG(4, 8, 256, 2)
    SMAP_PTG(4, 8, 256, 8)
    SMAP_PTG(4, 4, 256, 8)
    SMAP_PTG(4, 4, 256, 16)
    SMAP_PTG(3, 16, 256, 2)
    SMAP_PTG(3, 8, 256, 4)
#undef SMAP_PT
#undef SMAP_PTG
    }
    return kEunsupported;
}

template <bool BB>
int dispatch_point(int op, int m, const TileCfg &tc, const Plan &P, dim3 grid, const void *in, void *out,
                   hipStream_t s)
{
    switch (op) {
    case OP_MAP: return dispatch_point_shape<OP_MAP, BB>(m, tc, P, grid, in, out, s);
    case OP_ACCUM: return dispatch_point_shape<OP_ACCUM, BB>(m, tc, P, grid, in, out, s);
    case OP_HITS: return dispatch_point_shape<OP_HITS, BB>(m, tc, P, grid, in, out, s);
    case OP_HASH: return dispatch_point_shape<OP_HASH, BB>(m, tc, P, grid, in, out, s);
    case OP_EDM:
        if (m != 2) return kEinval;
        if (tc.grp != 1) return kEunsupported;       // one tile per workgroup only
        switch (tc.rho) {
        case 32: launch_point<2, 32, 256, 1, OP_EDM, BB>(P, grid, in, out, s); return kOk;
        case 16: launch_point<2, 16, 64, 1, OP_EDM, BB>(P, grid, in, out, s); return kOk;
        case 64: launch_point<2, 64, 256, 1, OP_EDM, BB>(P, grid, in, out, s); return kOk;
        case 128: launch_point<2, 128, 256, 2, OP_EDM, BB>(P, grid, in, out, s); return kOk;
        }
        return kEunsupported;
    }
    return kEinval;
}

template <int RHO, int RY, int RZ, int RL, bool BB>
void launch_ca3(const Plan &PL, dim3 grid, const uint8_t *in, uint8_t *out, hipStream_t s)
{
    constexpr int NT = Ca3Walk<RHO, RY, RZ, RL>::NT;
    if (PL.n < 15)
        hipLaunchKernelGGL((k_ca3<RHO, RY, RZ, RL, BB, true>), grid, dim3(NT), 0, s, PL, in, out);
    else
        hipLaunchKernelGGL((k_ca3<RHO, RY, RZ, RL, BB, false>), grid, dim3(NT), 0, s, PL, in, out);
}

template <bool BB>
int dispatch(int m, int op, const TileCfg &tc, const Plan &P0, const void *in, void *out,
             hipStream_t s)
{
    dim3 grid;
    const Plan &P = P0;  // grid and plan checks
    const uint32_t sub = (uint32_t)tc.sub;
    const uint32_t grp = (uint32_t)tc.grp;   // > 1 only for the pointwise ops (then sub = 1)
    if (BB) {
        const uint32_t kb = (uint32_t)P.kbox;
        const uint32_t kx = (kb + grp - 1) / grp;
        if (op == OP_CA2)
            grid = dim3(kb, kb * sub, 1);
        else
            grid = (m == 2) ? dim3(kx, kb, sub) : (m == 3 ? dim3(kx, kb, kb * sub) : dim3(kx, kb, kb * kb * sub));
    } else {
        grid = (op == OP_CA3) ? dim3(P.total, sub, 1) : dim3((P.total + grp - 1) / grp * sub, 1, 1);
    }
    Plan PL = P0;  // the kernels renumber workgroups over this grid
    PL.grid[0] = grid.x;
    PL.grid[1] = grid.y;
    PL.grid[2] = grid.z;
    PL.nwg = grid.x * grid.y * grid.z;
    PL.grid_div[0] = make_divu(grid.x);
    PL.grid_div[1] = make_divu(grid.y);
    // H runs XCD-contiguous (its workgroups are nearly all useful, so every
    // XCD gets an equal share of the work) when neighbouring tiles share
    // cache lines: the pointwise ops that touch memory.  Measured faster in
    // the hardware order: MAP (no memory traffic to share) and the automata
    // (their sub-block order already spreads the concurrent workgroups over
    // the buffer; 2-D: 66.8 against 69.6 us at n = 16384).  BB never splits
    // contiguously (the XCDs at the end of the range would get mostly empty
    // box tiles).  For the automata it scatters each group of 8 ids over
    // the XCDs: the plain order ties the useful tile columns to a few XCDs
    // when the box side shares a factor with 8 (3-D, n = 768-1023: 248-329
    // against 106-172 us).  The pointwise ops keep the plain order (4-D
    // hash: 29.9 against 34.7 us scattered).
    PL.remap = BB ? ((op == OP_CA2 || op == OP_CA3) ? 2u : 0u)
                  : ((op == OP_CA2 || op == OP_CA3 || op == OP_MAP) ? 0u : 1u);
    if (op == OP_CA2) {
        const uint8_t *i8 = (const uint8_t *)in;
        uint8_t *o8 = (uint8_t *)out;
        constexpr int D = 2;  // rows per block; two blocks in flight per wave
        switch (tc.rho * 10000 + tc.wg) {
#define SMAP_CA2(RHO, WG, W, R, WX)                                                              \
        case RHO * 10000 + WG:                                                                    \
            static_assert(Ca2Walk<RHO, W, R, WX>::SUB > 0, "shape");                              \
            if (P.n < 15)                                                                         \
                hipLaunchKernelGGL((k_ca2<RHO, W, R, D, BB, true, WX>), grid, dim3(WG), 0, s, PL, i8, o8); \
            else                                                                                  \
                hipLaunchKernelGGL((k_ca2<RHO, W, R, D, BB, false, WX>), grid, dim3(WG), 0, s, PL, i8, o8); \
            return kOk;
        SMAP_CA2(1024, 64, 1, 4, 1)
        SMAP_CA2(1024, 128, 2, 16, 1)
        SMAP_CA2(1024, 256, 4, 16, 1)
        SMAP_CA2(512, 512, 8, 16, 1)
        SMAP_CA2(256, 256, 4, 16, 1)
        SMAP_CA2(128, 128, 2, 8, 1)
        SMAP_CA2(2048, 128, 2, 16, 2)
        SMAP_CA2(2048, 256, 4, 16, 2)
        SMAP_CA2(4096, 256, 4, 16, 4)
#undef SMAP_CA2
        }
        return kEunsupported;
    }
    if (op == OP_CA3) {
        const uint8_t *i8 = (const uint8_t *)in;
        uint8_t *o8 = (uint8_t *)out;
        switch (tc.rho * 10000 + tc.wg) {
#define SMAP_CA3(RHO, WG, RY, RZ, RL)                                                             \
        case RHO * 10000 + WG:                                                                    \
            static_assert(Ca3Walk<RHO, RY, RZ, RL>::NT == WG, "CA3 shape");                      \
            launch_ca3<RHO, RY, RZ, RL, BB>(PL, grid, i8, o8, s);                                 \
            return kOk;
        SMAP_CA3(128, 256, 32, ca3_rz(128), 1)
        SMAP_CA3(128, 128, 16, ca3_rz(128), 1)
        SMAP_CA3(128, 512, 64, ca3_rz(128), 1)
        SMAP_CA3(256, 256, 16, ca3_rz(256), 1)
        SMAP_CA3(256, 128, 8, ca3_rz(256), 1)
        SMAP_CA3(256, 512, 32, ca3_rz(256), 1)
        SMAP_CA3(64, 128, 64, ca3_rz(64), 2)
        SMAP_CA3(64, 256, 64, ca3_rz(64), 1)
        SMAP_CA3(32, 64, 32, ca3_rz(32), 1)
#undef SMAP_CA3
        }
        return kEunsupported;
    }
    return dispatch_point<BB>(op, m, tc, PL, grid, in, out, s);
}

// The pieces of an H launch as concurrent launches: one stream per piece
// (created once per device, default priority), joined to the caller's
// stream through events.  g_piece_mu keeps one launch's record/wait
// sequence together.
struct PieceStreams {
    hipStream_t s[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t start = nullptr;
    hipEvent_t done[4] = {nullptr, nullptr, nullptr, nullptr};
};
std::mutex g_piece_mu;
std::map<int, PieceStreams> g_piece_streams;

int piece_streams_for_device(PieceStreams **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kEhip;
    PieceStreams &S = g_piece_streams[dev];
    if (!S.start) {
        for (int i = 0; i < 4; ++i) {
            if (hipStreamCreateWithFlags(&S.s[i], hipStreamNonBlocking) != hipSuccess) return kEhip;
            if (hipEventCreateWithFlags(&S.done[i], hipEventDisableTiming) != hipSuccess) return kEhip;
        }
        if (hipEventCreateWithFlags(&S.start, hipEventDisableTiming) != hipSuccess) return kEhip;
    }
    *out = &S;
    return kOk;
}

int launch_pieces(int m, int op, const TileCfg &tc, const Plan &P, const void *in, void *out, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_piece_mu);
    PieceStreams *S = nullptr;
    int rc = piece_streams_for_device(&S);
    if (rc != kOk) return rc;
    if (hipEventRecord(S->start, s) != hipSuccess) return kEhip;
    for (int p = 0; p < P.npieces; ++p) {
        Plan Q = P;
        Q.wg_base = P.piece_start[p];
        Q.total = P.piece_start[p + 1] - P.piece_start[p];
        if (hipStreamWaitEvent(S->s[p], S->start, 0) != hipSuccess) return kEhip;
        if (Q.total > 0) {
            rc = dispatch<false>(m, op, tc, Q, in, out, S->s[p]);
            if (rc != kOk) return rc;
        }
        if (hipEventRecord(S->done[p], S->s[p]) != hipSuccess) return kEhip;
    }
    for (int p = 0; p < P.npieces; ++p)
        if (hipStreamWaitEvent(s, S->done[p], 0) != hipSuccess) return kEhip;
    return kOk;
}

int do_launch(int m, int64_t n, int r, int beta, int op, const void *in, void *out,
              void *stream, bool bb)
{
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    int b = 0;
    if (!bb) {
        if (beta == 0) {  // a tuned beta, if any
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_tuned.find(std::make_tuple(m, n, op_class(op)));
            if (it != g_tuned.end()) beta = it->second.beta;
        }
        rc = resolve_rb(m, r, beta, &b);
        if (rc != kOk) return rc;
    }
    rc = check_buffers(m, n, op, in, out);
    if (rc != kOk) return rc;
    Plan P;
    TileCfg tc;
    rc = get_plan(m, n, b, op, bb, &P, nullptr, &tc);
    if (rc != kOk) return rc;
    if (P.total == 0) return kOk;
    hipStream_t s = (hipStream_t)stream;
    int general = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        general = g_general;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (general == 1 && hipStreamIsCapturing(s, &cap) != hipSuccess) return kEhip;
    if (!bb && general == 1 && P.npieces > 1 && cap == hipStreamCaptureStatusNone)
        rc = launch_pieces(m, op, tc, P, in, out, s);
    else
        rc = bb ? dispatch<true>(m, op, tc, P, in, out, s) : dispatch<false>(m, op, tc, P, in, out, s);
    if (rc != kOk) return rc;
    return hipGetLastError() == hipSuccess ? kOk : kEhip;
}

// ---- batched launches ------------------------------------------------------

// Batched tile shapes: CA2 rho 256 (4 waves, 16 rows per segment, one
// workgroup per tile); CA3 rho 64 (128 threads, 64 rows, 16 planes per
// sub-block, 2 rows per lane).
constexpr TileCfg kBatchCa2 = {256, 256, 1};
constexpr int kBatchCa3Ry = 64, kBatchCa3Rz = 16, kBatchCa3Rl = 2;
constexpr TileCfg kBatchCa3 = {64, 128, (64 / kBatchCa3Ry) * (64 / kBatchCa3Rz)};
constexpr int kBatchMaxJobs = 4096;   // jobs per launch (table capacity)

// Job tables live in a byte ring: pinned host staging plus a device copy of
// the same size.  A launch takes the bytes it needs (the prefix array,
// padded to 256 bytes, then the BatchJob array) right after the previous
// one, wrapping to the start; each use is released when the event recorded
// after its launch has completed.  Only when the ring is full does a launch
// wait, on the host, for the oldest use.
constexpr size_t kRingBytes = size_t(32) << 20;
// Two zeroed 8 KiB buffers after the ring: input and output of the warm-up
// steps of the serving loop (a 16^3 box each).
constexpr size_t kWarmBytes = 16384;

struct BatchRing {
    struct Use {
        size_t begin, end;
        hipEvent_t ev;
    };
    uint8_t *host = nullptr;
    uint8_t *dev = nullptr;    // kRingBytes of tables, then kWarmBytes of zeros
    size_t head = 0;
    std::deque<Use> used;            // in allocation (ring) order
    std::vector<hipEvent_t> spare;   // completed events for reuse
};
std::mutex g_batch_mu;
std::map<int, BatchRing> g_rings;  // per device

int ring_for_device(BatchRing **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kEhip;
    BatchRing &R = g_rings[dev];
    if (!R.dev) {
        if (hipHostMalloc((void **)&R.host, kRingBytes, hipHostMallocDefault) != hipSuccess) return kEhip;
        if (hipMalloc((void **)&R.dev, kRingBytes + kWarmBytes) != hipSuccess) {
            (void)hipHostFree(R.host);
            R.host = nullptr;
            return kEhip;
        }
        if (hipMemset(R.dev + kRingBytes, 0, kWarmBytes) != hipSuccess) return kEhip;
    }
    *out = &R;
    return kOk;
}

// Reserve `bytes` (a multiple of 256) of the ring at *off.
int ring_reserve(BatchRing &R, size_t bytes, size_t *off)
{
    if (bytes > kRingBytes) return kErange;
    const size_t a = (R.head + bytes > kRingBytes) ? 0 : R.head;
    for (;;) {
        // release finished uses, oldest first
        while (!R.used.empty()) {
            const hipError_t q = hipEventQuery(R.used.front().ev);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return kEhip;
            R.spare.push_back(R.used.front().ev);
            R.used.pop_front();
        }
        bool overlap = false;
        for (const BatchRing::Use &u : R.used) overlap = overlap || (u.begin < a + bytes && a < u.end);
        if (!overlap) break;
        // ring full here: wait for the oldest use (uses end in issue order of
        // their events on the host; waiting on the oldest first is enough)
        if (hipEventSynchronize(R.used.front().ev) != hipSuccess) return kEhip;
        R.spare.push_back(R.used.front().ev);
        R.used.pop_front();
    }
    *off = a;
    return kOk;
}

struct BatchItem {
    Plan P;
    const uint8_t *in;
    uint8_t *out;
    uint32_t nwg;  // workgroups of the job
};

// One launch of a kernel class over items[0..cnt): fill ring bytes, copy
// them to the device, launch, and mark the use with an event.
int launch_batch_chunk(BatchRing &R, int kind, const BatchItem *items, int cnt, hipStream_t s)
{
    const size_t start_bytes = ((sizeof(uint32_t) * (size_t)(cnt + 1) + 255) / 256) * 256;
    const size_t bytes = ((start_bytes + sizeof(BatchJob) * (size_t)cnt + 255) / 256) * 256;
    uint64_t acc = 0;
    for (int i = 0; i < cnt; ++i) acc += items[i].nwg;
    if (acc == 0) return kOk;
    if (acc > kMaxWorkgroups) return kErange;
    size_t off = 0;
    int rc = ring_reserve(R, bytes, &off);
    if (rc != kOk) return rc;
    uint8_t *h = R.host + off;
    uint8_t *d = R.dev + off;
    uint32_t *start = reinterpret_cast<uint32_t *>(h);
    BatchJob *jobs = reinterpret_cast<BatchJob *>(h + start_bytes);
    acc = 0;
    for (int i = 0; i < cnt; ++i) {
        start[i] = (uint32_t)acc;
        jobs[i].P = items[i].P;
        jobs[i].in = items[i].in;
        jobs[i].out = items[i].out;
        acc += items[i].nwg;
    }
    start[cnt] = (uint32_t)acc;
    if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return kEhip;
    const uint32_t *dstart = reinterpret_cast<const uint32_t *>(d);
    const BatchJob *djobs = reinterpret_cast<const BatchJob *>(d + start_bytes);
    const uint32_t nwg = (uint32_t)acc, nj = (uint32_t)cnt;
    switch (kind) {
    case 0:
        hipLaunchKernelGGL((k_ca2_batch<256, 4, 16, 2, false>), dim3(nwg), dim3(256), 0, s, dstart, djobs, nj, nwg);
        break;
    case 1:
        hipLaunchKernelGGL((k_ca2_batch<256, 4, 16, 2, true>), dim3(nwg), dim3(256), 0, s, dstart, djobs, nj, nwg);
        break;
    case 2:
        hipLaunchKernelGGL((k_ca3_batch<64, kBatchCa3Ry, kBatchCa3Rz, kBatchCa3Rl, false>), dim3(nwg),
                           dim3(kBatchCa3.wg), 0, s, dstart, djobs, nj, nwg);
        break;
    default:
        hipLaunchKernelGGL((k_ca3_batch<64, kBatchCa3Ry, kBatchCa3Rz, kBatchCa3Rl, true>), dim3(nwg),
                           dim3(kBatchCa3.wg), 0, s, dstart, djobs, nj, nwg);
        break;
    }
    if (hipGetLastError() != hipSuccess) return kEhip;
    hipEvent_t ev = nullptr;
    if (!R.spare.empty()) {
        ev = R.spare.back();
        R.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        return kEhip;
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        R.spare.push_back(ev);
        return kEhip;
    }
    R.used.push_back(BatchRing::Use{off, off + bytes, ev});
    R.head = off + bytes;
    return kOk;
}

// Workgroups of the queue kernel the device holds at once (occupancy times
// compute units), per device.
std::map<int, uint32_t> g_queue_grid;

int queue_grid_for_device(uint32_t *grid)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kEhip;
    auto it = g_queue_grid.find(dev);
    if (it == g_queue_grid.end()) {
        int cus = 0, occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return kEhip;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_queue),
                                                         kQueueThreads, 0) != hipSuccess)
            return kEhip;
        it = g_queue_grid.emplace(dev, (uint32_t)std::max(1, cus * std::max(1, occ))).first;
    }
    *grid = it->second;
    return kOk;
}

// Load the batched kernels' code and allocate the table ring before the
// first batch (both take milliseconds on first use).
int batch_prepare()
{
    hipFuncAttributes a;
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_ca2_batch<256, 4, 16, 2, false>),
        reinterpret_cast<const void *>(&k_ca2_batch<256, 4, 16, 2, true>),
        reinterpret_cast<const void *>(&k_ca3_batch<64, kBatchCa3Ry, kBatchCa3Rz, kBatchCa3Rl, false>),
        reinterpret_cast<const void *>(&k_ca3_batch<64, kBatchCa3Ry, kBatchCa3Rz, kBatchCa3Rl, true>),
        reinterpret_cast<const void *>(&k_queue),
    };
    for (const void *f : fns) {
        if (hipFuncGetAttributes(&a, f) != hipSuccess) return kEhip;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);   // and allocate the table ring now
    BatchRing *R = nullptr;
    const int rc = ring_for_device(&R);
    if (rc != kOk) return rc;
    uint32_t grid = 0;
    return queue_grid_for_device(&grid);
}

// The warm-up buffers of this device (allocated with the ring).
int warm_buffers(uint8_t **buf)
{
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchRing *R = nullptr;
    const int rc = ring_for_device(&R);
    if (rc == kOk) *buf = R->dev + kRingBytes;
    return rc;
}

int batch_launch(const simplex_job *jobs, int32_t njobs, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs)) return kEinval;
    if (njobs == 0) return kOk;
    // kinds: 0 CA2, 1 CA2 (n < 15), 2 CA3, 3 CA3 (n < 15)
    std::vector<BatchItem> items[4];
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int32_t i = 0; i < njobs; ++i) {
            const simplex_job &J = jobs[i];
            const bool ca2 = J.m == 2 && J.op == OP_CA2, ca3 = J.m == 3 && J.op == OP_CA3;
            if (!ca2 && !ca3) return kEinval;
            int rc = check_op(J.m, J.n, J.op);
            if (rc != kOk) return rc;
            rc = check_buffers(J.m, J.n, J.op, J.buf_in, J.buf_out);
            if (rc != kOk) return rc;
            const TileCfg &t = ca2 ? kBatchCa2 : kBatchCa3;
            BatchItem it{};
            rc = plan_for(J.m, J.n, 2, false, ca2 ? 1 : 2, t, &it.P, nullptr);
            if (rc != kOk) return rc;
            it.in = (const uint8_t *)J.buf_in;
            it.out = (uint8_t *)J.buf_out;
            it.nwg = it.P.total * (uint32_t)t.sub;
            items[(ca2 ? 0 : 2) + (J.n < 15 ? 1 : 0)].push_back(it);
        }
    }
    {
        const int rc = check_batch_buffers(jobs, njobs);
        if (rc != kOk) return rc;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchRing *R = nullptr;
    int rc = ring_for_device(&R);
    if (rc != kOk) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int kind = 0; kind < 4; ++kind) {
        const std::vector<BatchItem> &v = items[kind];
        for (size_t o = 0; o < v.size(); o += kBatchMaxJobs) {
            const int cnt = (int)std::min<size_t>(kBatchMaxJobs, v.size() - o);
            rc = launch_batch_chunk(*R, kind, v.data() + o, cnt, s);
            if (rc != kOk) return rc;
        }
    }
    return kOk;
}

// ---- persistent work-queue launch -----------------------------------------

// One persistent launch over items[0..cnt) (mixed kinds): ring bytes hold
// the head counter (zero), the unit prefix sums and the job array.
int launch_queue_chunk(BatchRing &R, const BatchItem *items, const uint32_t *kinds, int cnt, uint32_t max_wg,
                       hipStream_t s)
{
    constexpr size_t head_bytes = 256;
    const size_t start_bytes = ((sizeof(uint32_t) * (size_t)(cnt + 1) + 255) / 256) * 256;
    const size_t bytes = ((head_bytes + start_bytes + sizeof(QueueJob) * (size_t)cnt + 255) / 256) * 256;
    uint64_t acc = 0;
    for (int i = 0; i < cnt; ++i) acc += items[i].nwg;
    if (acc == 0) return kOk;
    if (acc > kMaxWorkgroups) return kErange;
    uint32_t grid = 0;
    int rc = queue_grid_for_device(&grid);
    if (rc != kOk) return rc;
    if (max_wg > 0) grid = std::min(grid, max_wg);
    grid = (uint32_t)std::min<uint64_t>(grid, acc);
    size_t off = 0;
    rc = ring_reserve(R, bytes, &off);
    if (rc != kOk) return rc;
    uint8_t *h = R.host + off;
    uint8_t *d = R.dev + off;
    std::memset(h, 0, head_bytes);
    uint32_t *start = reinterpret_cast<uint32_t *>(h + head_bytes);
    QueueJob *jobs = reinterpret_cast<QueueJob *>(h + head_bytes + start_bytes);
    acc = 0;
    for (int i = 0; i < cnt; ++i) {
        start[i] = (uint32_t)acc;
        jobs[i].P = items[i].P;
        jobs[i].in = items[i].in;
        jobs[i].out = items[i].out;
        jobs[i].kind = kinds[i];
        jobs[i].reserved = 0;
        acc += items[i].nwg;
    }
    start[cnt] = (uint32_t)acc;
    if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return kEhip;
    hipLaunchKernelGGL(k_queue, dim3(grid), dim3(kQueueThreads), 0, s, reinterpret_cast<uint32_t *>(d),
                       reinterpret_cast<const uint32_t *>(d + head_bytes),
                       reinterpret_cast<const QueueJob *>(d + head_bytes + start_bytes), (uint32_t)cnt,
                       (uint32_t)acc);
    if (hipGetLastError() != hipSuccess) return kEhip;
    hipEvent_t ev = nullptr;
    if (!R.spare.empty()) {
        ev = R.spare.back();
        R.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        return kEhip;
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        R.spare.push_back(ev);
        return kEhip;
    }
    R.used.push_back(BatchRing::Use{off, off + bytes, ev});
    R.head = off + bytes;
    return kOk;
}

// Validated work items of the queue kernel for jobs[0..njobs) (g_mu taken here).
int queue_items(const simplex_job *jobs, int32_t njobs, std::vector<BatchItem> &items,
                std::vector<uint32_t> &kinds)
{
    constexpr TileCfg kQ2 = {kQueueCa2Rho, kQueueThreads, 1};
    constexpr TileCfg kQ3 = {kQueueCa3Rho, kQueueThreads,
                             (kQueueCa3Rho / kQueueCa3Ry) * (kQueueCa3Rho / kQueueCa3Rz)};
    static_assert(Ca2Walk<kQueueCa2Rho, kQueueCa2W, kQueueCa2R>::SUB == kQ2.sub &&
                  Ca3Walk<kQueueCa3Rho, kQueueCa3Ry, kQueueCa3Rz, kQueueCa3Rl>::SUB == kQ3.sub,
                  "queue tile configurations disagree with the kernel");
    items.clear();
    kinds.clear();
    items.reserve((size_t)njobs);
    kinds.reserve((size_t)njobs);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int32_t i = 0; i < njobs; ++i) {
            const simplex_job &J = jobs[i];
            const bool ca2 = J.m == 2 && J.op == OP_CA2, ca3 = J.m == 3 && J.op == OP_CA3;
            if (!ca2 && !ca3) return kEinval;
            int rc = check_op(J.m, J.n, J.op);
            if (rc != kOk) return rc;
            rc = check_buffers(J.m, J.n, J.op, J.buf_in, J.buf_out);
            if (rc != kOk) return rc;
            const TileCfg &t = ca2 ? kQ2 : kQ3;
            BatchItem it{};
            rc = plan_for(J.m, J.n, 2, false, ca2 ? 1 : 2, t, &it.P, nullptr);
            if (rc != kOk) return rc;
            it.in = (const uint8_t *)J.buf_in;
            it.out = (uint8_t *)J.buf_out;
            const bool small = J.n < kQueueSmallN;
            it.nwg = small ? 1u : it.P.total * (uint32_t)t.sub;   // a small job is one unit
            items.push_back(it);
            kinds.push_back(small ? (ca2 ? kQueueCa2Small : kQueueCa3Small) : (ca2 ? kQueueCa2 : kQueueCa3));
        }
    }
    return check_batch_buffers(jobs, njobs);
}

// The device-side table of one queue launch: head counter (zero), unit
// prefix sums, jobs.  Returns its size; fills `h` (bytes, 256-aligned
// sections) and the offsets of its parts.
size_t queue_table(const BatchItem *items, const uint32_t *kinds, int cnt, std::vector<uint8_t> &h,
                   size_t *start_off, size_t *jobs_off, uint64_t *units)
{
    constexpr size_t head_bytes = 256;
    const size_t start_bytes = ((sizeof(uint32_t) * (size_t)(cnt + 1) + 255) / 256) * 256;
    const size_t bytes = ((head_bytes + start_bytes + sizeof(QueueJob) * (size_t)cnt + 255) / 256) * 256;
    h.assign(bytes, 0);
    uint32_t *start = reinterpret_cast<uint32_t *>(h.data() + head_bytes);
    QueueJob *jobs = reinterpret_cast<QueueJob *>(h.data() + head_bytes + start_bytes);
    uint64_t acc = 0;
    for (int i = 0; i < cnt; ++i) {
        start[i] = (uint32_t)acc;
        jobs[i].P = items[i].P;
        jobs[i].in = items[i].in;
        jobs[i].out = items[i].out;
        jobs[i].kind = kinds[i];
        jobs[i].reserved = 0;
        acc += items[i].nwg;
    }
    start[cnt] = (uint32_t)acc;
    *start_off = head_bytes;
    *jobs_off = head_bytes + start_bytes;
    *units = acc;
    return bytes;
}

int queue_launch(const simplex_job *jobs, int32_t njobs, int32_t max_wg, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs) || max_wg < 0) return kEinval;
    if (njobs == 0) return kOk;
    std::vector<BatchItem> items;
    std::vector<uint32_t> kinds;
    int rc = queue_items(jobs, njobs, items, kinds);
    if (rc != kOk) return rc;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchRing *R = nullptr;
    rc = ring_for_device(&R);
    if (rc != kOk) return rc;
    for (size_t o = 0; o < items.size(); o += kBatchMaxJobs) {
        const int cnt = (int)std::min<size_t>(kBatchMaxJobs, items.size() - o);
        rc = launch_queue_chunk(*R, items.data() + o, kinds.data() + o, cnt, (uint32_t)max_wg,
                                (hipStream_t)stream);
        if (rc != kOk) return rc;
    }
    return kOk;
}

// ---- persistent launch without allocation ---------------------------------

// The job table of simplex_queue_launch_static lives in this file-scope
// device array (one copy per device, held until the process ends): the head
// counter, the unit prefix sums and the jobs, laid out as queue_table does.
constexpr int32_t kStaticMaxJobs = 256;
constexpr size_t kStaticBytes = 256 + ((sizeof(uint32_t) * (kStaticMaxJobs + 1) + 255) / 256) * 256 +
                                ((sizeof(QueueJob) * kStaticMaxJobs + 255) / 256) * 256;
__device__ __align__(256) uint8_t scratch[kStaticBytes];

// Per device: the device address of `scratch` (from hipGetSymbolAddress;
// the array's name is not a device address in host code), a host staging
// copy of the table (pageable; the copy reads it), and an event recorded
// after the last copy, so the staging bytes are rewritten only after the
// previous copy has read them.
struct StaticTable {
    uint8_t *dev = nullptr;
    std::vector<uint8_t> stage;
    hipEvent_t copied = nullptr;
    bool pending = false;
};
std::mutex g_static_mu;
std::map<int, StaticTable> g_static;

int static_table_for_device(StaticTable **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kEhip;
    StaticTable &T = g_static[dev];
    if (!T.dev) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return kEhip;
        if (!T.copied && hipEventCreateWithFlags(&T.copied, hipEventDisableTiming) != hipSuccess) return kEhip;
        T.stage.assign(kStaticBytes, 0);
        T.dev = static_cast<uint8_t *>(p);
    }
    *out = &T;
    return kOk;
}

int queue_launch_static(const simplex_job *jobs, int32_t njobs, int32_t max_wg, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs) || max_wg < 0) return kEinval;
    if (njobs > kStaticMaxJobs) return kErange;
    if (njobs == 0) return kOk;
    std::vector<BatchItem> items;
    std::vector<uint32_t> kinds;
    int rc = queue_items(jobs, njobs, items, kinds);
    if (rc != kOk) return rc;
    std::vector<uint8_t> h;
    size_t start_off = 0, jobs_off = 0;
    uint64_t units = 0;
    const size_t bytes = queue_table(items.data(), kinds.data(), njobs, h, &start_off, &jobs_off, &units);
    if (bytes > kStaticBytes) return kErange;
    if (units == 0) return kOk;
    if (units > kMaxWorkgroups) return kErange;
    uint32_t grid = 0;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        rc = queue_grid_for_device(&grid);
    }
    if (rc != kOk) return rc;
    if (max_wg > 0) grid = std::min(grid, (uint32_t)max_wg);
    grid = (uint32_t)std::min<uint64_t>(grid, units);
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticTable *T = nullptr;
    rc = static_table_for_device(&T);
    if (rc != kOk) return rc;
    // the previous copy out of the staging bytes has finished before they change
    if (T->pending && hipEventSynchronize(T->copied) != hipSuccess) return kEhip;
    std::memcpy(T->stage.data(), h.data(), bytes);      // head counter included: starts at zero
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(T->dev, T->stage.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess) return kEhip;
    if (hipEventRecord(T->copied, s) != hipSuccess) return kEhip;
    T->pending = true;
    hipLaunchKernelGGL(k_queue, dim3(grid), dim3(kQueueThreads), 0, s, reinterpret_cast<uint32_t *>(T->dev),
                       reinterpret_cast<const uint32_t *>(T->dev + start_off),
                       reinterpret_cast<const QueueJob *>(T->dev + jobs_off), (uint32_t)njobs, (uint32_t)units);
    return hipGetLastError() == hipSuccess ? kOk : kEhip;
}

// ---- autotuning -----------------------------------------------------------

// The compiled (rho, threads) choices of (m, op class).
std::vector<TileCfg> tile_candidates(int m, int cls)
{
    std::vector<TileCfg> v;
    if (cls == 0) {
        for (const PointShape &c : kPointShapes)
            if (c.m == m) v.push_back({c.rho, c.wg, c.sub, c.grp});
    } else if (cls == 1) {
        for (const Ca2Shape &c : kCa2Shapes) v.push_back({c.rho, c.wg, c.sub});
    } else {
        for (const Ca3Shape &c : kCa3Shapes) v.push_back({c.rho, c.wg, c.sub});
    }
    return v;
}

bool device_key(char *buf, size_t len)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    char arch[64];
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char *c = arch; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    std::snprintf(buf, len, "%s_%dcu", arch, prop.multiProcessorCount);
    return true;
}

bool cache_lookup(const char *path, const char *dev, int m, int64_t n, int op, simplex_tune_result *r)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256], d[96];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int mm, oo, rho, wg, beta, grp;
        long long nn;
        float us;
        if (std::sscanf(line, "smap-tune-v2 %95s %d %lld %d %d %d %d %d %f", d, &mm, &nn, &oo, &rho, &wg, &grp, &beta,
                        &us) == 9 &&
            std::strcmp(d, dev) == 0 && mm == m && nn == n && oo == op) {
            *r = simplex_tune_result{rho, wg, beta, us, grp};
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

int autotune(int m, int64_t n, int op, const void *in, void *out, int32_t reps, const char *cache_path,
             void *stream, simplex_tune_result *best)
{
    if (!best || reps < 1) return kEinval;
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    rc = check_buffers(m, n, op, in, out);
    if (rc != kOk) return rc;
    if (op == OP_ACCUM && in == out) return kEinval;
    const int cls = op_class(op);
    const auto key = std::make_tuple(m, n, cls);
    char dev[96] = "unknown";
    if (!device_key(dev, sizeof dev)) return kEhip;
    simplex_tune_result r{};
    if (cache_path && cache_lookup(cache_path, dev, m, n, op, &r)) {
        int wg = r.wg_threads, sub = 1, grp = r.tiles_per_wg;
        if (tile_supported(m, cls, r.rho, &wg, &sub, &grp)) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_tuned[key] = Tuned{{r.rho, wg, sub, grp}, r.beta};
            *best = r;
            return kOk;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return kEhip;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return kEhip;
    }
    const std::vector<int> betas = m == 4 ? std::vector<int>{3, 4} : std::vector<int>{2};
    simplex_tune_result top{0, 0, 0, 0.f, 1};
    bool have = false;
    rc = kOk;
    for (const TileCfg &t : tile_candidates(m, cls)) {
        for (int beta : betas) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_tuned[key] = Tuned{t, beta};
            }
            int lr = kOk;
            for (int i = 0; i < 2 && lr == kOk; ++i) lr = do_launch(m, n, 0, beta, op, in, out, stream, false);
            if (lr == kErange || lr == kEunsupported) continue;  // not for this size or op
            if (lr != kOk) { rc = lr; break; }
            if (hipEventRecord(e0, s) != hipSuccess) { rc = kEhip; break; }
            for (int i = 0; i < reps && lr == kOk; ++i) lr = do_launch(m, n, 0, beta, op, in, out, stream, false);
            if (lr != kOk) { rc = lr; break; }
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = kEhip; break; }
            const float us = ms * 1e3f / (float)reps;
            if (!have || us < top.us) top = simplex_tune_result{t.rho, t.wg, beta, us, t.grp};
            have = true;
        }
        if (rc != kOk) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_mu);
    if (rc != kOk || !have) {
        g_tuned.erase(key);
        return rc != kOk ? rc : kErange;
    }
    int wg = top.wg_threads, sub = 1, grp = top.tiles_per_wg;
    tile_supported(m, cls, top.rho, &wg, &sub, &grp);
    g_tuned[key] = Tuned{{top.rho, wg, sub, grp}, top.beta};
    *best = top;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (!f) return kEinval;
        std::fprintf(f, "smap-tune-v2 %s %d %lld %d %d %d %d %d %.3f\n", dev, m, (long long)n, op, top.rho,
                     top.wg_threads, top.tiles_per_wg, top.beta, top.us);
        std::fclose(f);
    }
    return kOk;
}

// ---- graphs --------------------------------------------------------------

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *table = nullptr;   // device memory the graph's kernels read (queue graphs)
};

// One persistent work-queue launch over a fixed job set, captured as a
// graph: a fill kernel clears the head counter (no memset node), then the
// queue kernel runs; the job table lives in device memory the graph owns.
int queue_graph_create(const simplex_job *jobs, int32_t njobs, int32_t max_wg, void **handle)
{
    if (!handle || njobs < 1 || !jobs || max_wg < 0) return kEinval;
    *handle = nullptr;
    if (njobs > kBatchMaxJobs) return kErange;
    std::vector<BatchItem> items;
    std::vector<uint32_t> kinds;
    int rc = queue_items(jobs, njobs, items, kinds);
    if (rc != kOk) return rc;
    std::vector<uint8_t> h;
    size_t start_off = 0, jobs_off = 0;
    uint64_t units = 0;
    const size_t bytes = queue_table(items.data(), kinds.data(), njobs, h, &start_off, &jobs_off, &units);
    if (units == 0) return kEinval;
    if (units > kMaxWorkgroups) return kErange;
    uint32_t grid = 0;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        rc = queue_grid_for_device(&grid);
    }
    if (rc != kOk) return rc;
    if (max_wg > 0) grid = std::min(grid, (uint32_t)max_wg);
    grid = (uint32_t)std::min<uint64_t>(grid, units);
    GraphHandle *gh = new GraphHandle();
    uint8_t *d = nullptr;
    if (hipMalloc((void **)&d, bytes) != hipSuccess) {
        delete gh;
        return kEhip;
    }
    gh->table = d;
    hipStream_t cs = nullptr;
    rc = kOk;
    if (hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) rc = kEhip;
    if (rc == kOk && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = kEhip;
    if (rc == kOk && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = kEhip;
    if (rc == kOk) {
        uint32_t *head = reinterpret_cast<uint32_t *>(d);
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, cs, head, 1u);
        hipLaunchKernelGGL(k_queue, dim3(grid), dim3(kQueueThreads), 0, cs, head,
                           reinterpret_cast<const uint32_t *>(d + start_off),
                           reinterpret_cast<const QueueJob *>(d + jobs_off), (uint32_t)njobs, (uint32_t)units);
        if (hipGetLastError() != hipSuccess) rc = kEhip;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc == kOk && e != hipSuccess) rc = kEhip;
        gh->graph = g;
        if (rc == kOk && hipGraphInstantiate(&gh->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = kEhip;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != kOk) {
        if (gh->exec) (void)hipGraphExecDestroy(gh->exec);
        if (gh->graph) (void)hipGraphDestroy(gh->graph);
        (void)hipFree(gh->table);
        delete gh;
        return rc;
    }
    *handle = gh;
    return kOk;
}

int graph_create(int m, int64_t n, int r, int beta, int op, bool bb, const void *in, void *out,
                 int32_t steps, void **handle)
{
    if (!handle || steps < 1) return kEinval;
    *handle = nullptr;
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    rc = check_buffers(m, n, op, in, out);
    if (rc != kOk) return rc;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return kEhip;
    GraphHandle *h = new GraphHandle();
    rc = kOk;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = kEhip;
    } else {
        const bool ca = op == OP_CA2 || op == OP_CA3;
        for (int32_t i = 0; i < steps && rc == kOk; ++i) {
            const void *a = (ca && (i & 1)) ? out : in;
            void *b = (ca && (i & 1)) ? const_cast<void *>(in) : out;
            rc = do_launch(m, n, r, beta, op, a, b, cs, bb);
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc == kOk && e != hipSuccess) rc = kEhip;
        h->graph = g;
        if (rc == kOk && hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = kEhip;
    }
    (void)hipStreamDestroy(cs);
    if (rc != kOk) {
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        delete h;
        return rc;
    }
    *handle = h;
    return kOk;
}

// ---- several generations per pass (CA2) ------------------------------------

constexpr int kStepsRho = 256, kStepsKh = 32;   // tile side and halo (= generations per pass)
constexpr TileCfg kStepsTile = {kStepsRho, Ca2kShape<kStepsRho, kStepsKh>::NT, 1};
// CA3: 64^3 tiles, 16-cell halo (16 generations per pass), one bit per cell
constexpr int kSteps3Rho = 64, kSteps3Kh = 16;
constexpr TileCfg kSteps3Tile = {kSteps3Rho, Ca3kShape<kSteps3Rho, kSteps3Kh>::NT, 1};

int steps_launch(int m, int64_t n, int r, int beta, int op, int32_t steps, void *a, void *b,
                 void *stream, bool bb)
{
    const bool ca3 = m == 3 && op == OP_CA3;
    if (!(m == 2 && op == OP_CA2) && !ca3) return (check_op(m, n, op) != kOk) ? kEinval : kEunsupported;
    if (steps < 1) return kEinval;
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    int bt = 0;
    if (!bb) {
        rc = resolve_rb(m, r, beta, &bt);
        if (rc != kOk) return rc;
    }
    rc = check_buffers(m, n, op, a, b);
    if (rc != kOk) return rc;
    Plan P;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rc = plan_for(m, n, bt, bb, ca3 ? 2 : 1, ca3 ? kSteps3Tile : kStepsTile, &P, nullptr, true);
    }
    if (rc != kOk) return rc;
    if (P.total == 0) return kOk;
    const uint32_t kb = (uint32_t)P.kbox;
    const dim3 grid = bb ? dim3(kb, kb, ca3 ? kb : 1) : dim3(P.total, 1, 1);
    P.grid[0] = grid.x;
    P.grid[1] = grid.y;
    P.grid[2] = grid.z;
    P.nwg = grid.x * grid.y * grid.z;
    P.grid_div[0] = make_divu(grid.x);
    P.grid_div[1] = make_divu(grid.y);
    P.remap = bb ? 2u : 1u;
    // passes of at most kStepsKh generations, alternating a -> b -> a ...;
    // an odd number of passes, so that the last one writes b
    const int kh = ca3 ? kSteps3Kh : kStepsKh;   // generations per pass at most
    int passes = (steps + kh - 1) / kh;
    if (passes % 2 == 0) ++passes;
    hipStream_t s = (hipStream_t)stream;
    int left = steps;
    for (int i = 0; i < passes; ++i) {
        const int g = (left + (passes - i) - 1) / (passes - i);   // spread evenly, 1..kh
        const uint8_t *src = (const uint8_t *)((i & 1) ? b : a);
        uint8_t *dst = (uint8_t *)((i & 1) ? a : b);
        const bool safe = n < 15;
        constexpr int nt3 = Ca3kShape<kSteps3Rho, kSteps3Kh>::NT;
        constexpr int nt2 = Ca2kShape<kStepsRho, kStepsKh>::NT;
        if (ca3) {
            if (bb) {
                if (safe) hipLaunchKernelGGL((k_ca3k<kSteps3Rho, kSteps3Kh, true, true>), grid, dim3(nt3), 0, s, P, src, dst, g);
                else hipLaunchKernelGGL((k_ca3k<kSteps3Rho, kSteps3Kh, true, false>), grid, dim3(nt3), 0, s, P, src, dst, g);
            } else {
                if (safe) hipLaunchKernelGGL((k_ca3k<kSteps3Rho, kSteps3Kh, false, true>), grid, dim3(nt3), 0, s, P, src, dst, g);
                else hipLaunchKernelGGL((k_ca3k<kSteps3Rho, kSteps3Kh, false, false>), grid, dim3(nt3), 0, s, P, src, dst, g);
            }
        } else if (bb) {
            if (safe) hipLaunchKernelGGL((k_ca2k<kStepsRho, kStepsKh, true, true>), grid, dim3(nt2), 0, s, P, src, dst, g);
            else hipLaunchKernelGGL((k_ca2k<kStepsRho, kStepsKh, true, false>), grid, dim3(nt2), 0, s, P, src, dst, g);
        } else {
            if (safe) hipLaunchKernelGGL((k_ca2k<kStepsRho, kStepsKh, false, true>), grid, dim3(nt2), 0, s, P, src, dst, g);
            else hipLaunchKernelGGL((k_ca2k<kStepsRho, kStepsKh, false, false>), grid, dim3(nt2), 0, s, P, src, dst, g);
        }
        if (hipGetLastError() != hipSuccess) return kEhip;
        left -= g;
    }
    return kOk;
}

}  // namespace

extern "C" {

int simplex_map_launch(int m, int64_t n, int r, int beta, int op, const void *buf_in,
                       void *buf_out, void *stream)
{
    return do_launch(m, n, r, beta, op, buf_in, buf_out, stream, false);
}

int simplex_bb_launch(int m, int64_t n, int op, const void *buf_in, void *buf_out, void *stream)
{
    return do_launch(m, n, 0, 0, op, buf_in, buf_out, stream, true);
}

int simplex_count(int m, int64_t n, uint64_t *out)
{
    if (m < 1 || m > 64 || n < 0 || !out) return kEinval;
    return binom_u64((uint64_t)n + (uint64_t)m, (uint64_t)m, out) ? kOk : kErange;
}

int simplex_plan_info(int m, int64_t n, int r, int beta, int op, int use_bb,
                      struct simplex_plan_info *out)
{
    if (!out) return kEinval;
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    int b = 0;
    if (!use_bb) {
        rc = resolve_rb(m, r, beta, &b);
        if (rc != kOk) return rc;
    }
    Plan P;
    PlanCounts C;
    TileCfg tc;
    rc = get_plan(m, n, b, op, use_bb != 0, &P, &C, &tc);
    if (rc != kOk) return rc;
    struct simplex_plan_info info{};
    info.m = m;
    info.use_bb = use_bb ? 1 : 0;
    info.n = n;
    info.r = use_bb ? 0 : 2;
    info.beta = use_bb ? 0 : b;
    info.rho = tc.rho;
    info.wg_threads = tc.wg;
    info.tile_side_k = P.K;
    info.native_n = use_bb ? 0 : (1 << P.j);
    info.shell_layers = use_bb ? 0 : P.L;
    info.n_pieces = use_bb ? 1 : P.npieces;
    if (!binom_u64((uint64_t)n + m, (uint64_t)m, &info.useful_elements)) return kErange;
    info.useful_tiles = C.useful_tiles;
    info.launched_tiles = C.launched;
    info.wgs_per_tile = tc.sub;
    info.tiles_per_wg = tc.grp;
    if (tc.grp > 1) {
        // H: consecutive map units; BB: rows of the tile grid cut along x_1
        const uint64_t kb = (uint64_t)P.kbox, g = (uint64_t)tc.grp;
        info.launched_wgs = use_bb ? (kb + g - 1) / g * (C.launched / kb) : (C.launched + g - 1) / g;
    } else {
        info.launched_wgs = C.launched * (uint64_t)tc.sub;
    }
    info.native_wgs = C.native;
    info.full_tiles = C.full_tiles;
    *out = info;
    return kOk;
}

int simplex_plan_tiles(int m, int64_t n, int r, int beta, int op, int use_bb, int32_t *tiles,
                       uint64_t cap, uint64_t *written)
{
    int rc = check_op(m, n, op);
    if (rc != kOk) return rc;
    int b = 0;
    if (!use_bb) {
        rc = resolve_rb(m, r, beta, &b);
        if (rc != kOk) return rc;
    }
    Plan P;
    TileCfg tc;
    rc = get_plan(m, n, b, op, use_bb != 0, &P, nullptr, &tc);
    if (rc != kOk) return rc;
    if (written) *written = P.total;
    if (!tiles) return kOk;
    const uint64_t cnt = P.total < cap ? P.total : cap;
    const uint32_t kb = (uint32_t)P.kbox;
    for (uint64_t w = 0; w < cnt; ++w) {
        int32_t t[4] = {0, 0, 0, 0};
        bool ok;
        if (use_bb) {
            const uint32_t gx = (uint32_t)(w % kb), gy = (uint32_t)((w / kb) % kb);
            const uint32_t gz = (uint32_t)(w / ((uint64_t)kb * kb));
            decode_bb(P, gx, gy, gz, t);
            int64_t s = 0;
            for (int k = 0; k < m; ++k) s += (int64_t)t[k] * tc.rho;
            ok = s <= n;
        } else {
            ok = decode_h_rt(P, (uint32_t)w, t);
        }
        int32_t *o = tiles + 5 * w;
        o[0] = ok ? 1 : 0;
        for (int k = 0; k < 4; ++k) o[1 + k] = ok ? t[k] : 0;
    }
    return kOk;
}

int simplex_set_shape(int m, int op, int rho, int wg_threads, int tiles_per_wg)
{
    int rc = check_op(m, 0, op);
    if (rc != kOk) return rc;
    if (wg_threads < 0 || tiles_per_wg < 0) return kEinval;
    const int cls = op_class(op);
    std::lock_guard<std::mutex> lk(g_mu);
    if (rho == 0) {
        g_tiles.erase({m, cls});
        return kOk;
    }
    int wg = wg_threads, sub = 1, grp = tiles_per_wg;
    if (!tile_supported(m, cls, rho, &wg, &sub, &grp)) return kEunsupported;
    g_tiles[{m, cls}] = TileCfg{rho, wg, sub, grp};
    return kOk;
}

int simplex_set_tile(int m, int op, int rho, int wg_threads)
{
    return simplex_set_shape(m, op, rho, wg_threads, 0);
}

int simplex_batch_launch(const struct simplex_job *jobs, int32_t njobs, void *stream)
{
    return batch_launch(jobs, njobs, stream);
}

int simplex_queue_launch(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups, void *stream)
{
    return queue_launch(jobs, njobs, max_workgroups, stream);
}

int simplex_queue_launch_static(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups,
                                void *stream)
{
    return queue_launch_static(jobs, njobs, max_workgroups, stream);
}

int simplex_serve_run(const struct simplex_serve_job *jobs, int32_t njobs, void *arena,
                      uint64_t arena_bytes, int32_t mode, int32_t max_inflight, int32_t keep_outputs,
                      struct simplex_serve_record *records)
{
    if (njobs < 0 || (njobs > 0 && (!jobs || !arena))) return kEinval;
    if (mode != SMAP_SERVE_SEQUENTIAL && mode != SMAP_SERVE_BATCHED && mode != SMAP_SERVE_PERSISTENT)
        return kEinval;
    if (mode != SMAP_SERVE_SEQUENTIAL && max_inflight < 1) return kEinval;
    uint64_t need_all = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        const simplex_serve_job &J = jobs[i];
        const bool ok = (J.m == 2 && J.op == OP_CA2) || (J.m == 3 && J.op == OP_CA3);
        if (!ok || J.n < 0 || !J.buf_in) return kEinval;
        if (!(J.arrival_s >= 0.0) || (i > 0 && J.arrival_s < jobs[i - 1].arrival_s)) return kEinval;
        int64_t elems;
        if (!box_elems(J.m, J.n, &elems)) return kErange;
        const uint64_t b = Arena::round((uint64_t)elems);
        if (b > (arena_bytes & ~uint64_t(255))) return kEinval;   // could never be admitted
        need_all += b;
    }
    if (keep_outputs && need_all > (arena_bytes & ~uint64_t(255))) return kEinval;
    if (njobs == 0) return kOk;
    std::vector<simplex_serve_record> local;
    if (!records) {
        local.resize((size_t)njobs);
        records = local.data();
    }
    for (int32_t i = 0; i < njobs; ++i) records[i] = simplex_serve_record{-1.0, -1.0, -1.0, -1.0, 0, -1, kOk};
    if (mode != SMAP_SERVE_SEQUENTIAL) {
        const int rc = batch_prepare();
        if (rc != kOk) return rc;
    }
    uint8_t *warm = nullptr;
    const int rc = warm_buffers(&warm);
    if (rc != kOk) return rc;
    return serve_run(jobs, njobs, (uint8_t *)arena, arena_bytes, mode, max_inflight, keep_outputs, records,
                     warm);
}

int simplex_autotune(int m, int64_t n, int op, const void *buf_in, void *buf_out, int32_t reps,
                     const char *cache_path, void *stream, struct simplex_tune_result *best)
{
    return autotune(m, n, op, buf_in, buf_out, reps, cache_path, stream, best);
}

int simplex_autotune_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned.clear();
    return kOk;
}

int simplex_graph_create(int m, int64_t n, int r, int beta, int op, int use_bb, const void *buf_in,
                         void *buf_out, int32_t steps, void **graph)
{
    return graph_create(m, n, r, beta, op, use_bb != 0, buf_in, buf_out, steps, graph);
}

int simplex_queue_graph_create(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups,
                               void **graph)
{
    return queue_graph_create(jobs, njobs, max_workgroups, graph);
}

int simplex_graph_launch(void *graph, void *stream)
{
    if (!graph) return kEinval;
    GraphHandle *h = static_cast<GraphHandle *>(graph);
    return hipGraphLaunch(h->exec, (hipStream_t)stream) == hipSuccess ? kOk : kEhip;
}

int simplex_graph_destroy(void *graph)
{
    if (!graph) return kOk;
    GraphHandle *h = static_cast<GraphHandle *>(graph);
    int rc = kOk;
    if (h->exec && hipGraphExecDestroy(h->exec) != hipSuccess) rc = kEhip;
    if (h->graph && hipGraphDestroy(h->graph) != hipSuccess) rc = kEhip;
    if (h->table && hipFree(h->table) != hipSuccess) rc = kEhip;
    delete h;
    return rc;
}

int simplex_map_launch_steps(int m, int64_t n, int r, int beta, int op, int32_t steps, void *buf_in,
                             void *buf_out, void *stream)
{
    return steps_launch(m, n, r, beta, op, steps, buf_in, buf_out, stream, false);
}

int simplex_bb_launch_steps(int m, int64_t n, int op, int32_t steps, void *buf_in, void *buf_out,
                            void *stream)
{
    return steps_launch(m, n, 0, 0, op, steps, buf_in, buf_out, stream, true);
}

int simplex_set_general(int strategy)
{
    if (strategy != SMAP_GENERAL_FUSED && strategy != SMAP_GENERAL_STREAMS) return kEinval;
    std::lock_guard<std::mutex> lk(g_mu);
    g_general = strategy;
    return kOk;
}

int simplex_set_layout(int m, int layout)
{
    if (m != 3 || (layout != SMAP_LAYOUT_AUTO && layout != SMAP_LAYOUT_PACKED && layout != SMAP_LAYOUT_LEVELS))
        return kEinval;
    std::lock_guard<std::mutex> lk(g_mu);
    g_layout3 = layout;
    return kOk;
}

int simplex_copy_launch(int m, int64_t n, const void *buf_in, void *buf_out, void *stream)
{
    if ((m != 2 && m != 3) || n < 0 || !buf_in || !buf_out) return kEinval;
    int64_t elems = 0;
    if (!box_elems(m, n, &elems)) return kErange;
    if (n + 1 > 65535 && m == 3) return kErange;                 // grid y is the slab
    const uintptr_t a = (uintptr_t)buf_in, b = (uintptr_t)buf_out;
    if (a < b + (uintptr_t)elems && b < a + (uintptr_t)elems) return kEinval;
    const dim3 grid((uint32_t)((n + kCopyRowsPerWg) / kCopyRowsPerWg), m == 3 ? (uint32_t)(n + 1) : 1u);
    hipStream_t s = (hipStream_t)stream;
    const uint8_t *i8 = (const uint8_t *)buf_in;
    uint8_t *o8 = (uint8_t *)buf_out;
    if (m == 2)
        hipLaunchKernelGGL(k_simplex_copy<2>, grid, dim3(256), 0, s, (int32_t)n, (int64_t)(n + 1), i8, o8);
    else
        hipLaunchKernelGGL(k_simplex_copy<3>, grid, dim3(256), 0, s, (int32_t)n, (int64_t)(n + 1), i8, o8);
    return hipGetLastError() == hipSuccess ? kOk : kEhip;
}

const char *simplex_strerror(int status)
{
    switch (status) {
    case SMAP_OK: return "success";
    case SMAP_EINVAL: return "invalid argument (m, n, op, pointer or overlapping buffers)";
    case SMAP_EUNSUPPORTED: return "unsupported (r, beta) or tile configuration";
    case SMAP_ERANGE: return "sizes exceed the supported index range";
    case SMAP_EHIP: return "the HIP runtime reported a launch error";
    }
    return "unknown status";
}

}  // extern "C"
