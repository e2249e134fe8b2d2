// Batched systems: one workgroup runs every step of one system.
//
// Parameter sweeps run many small, independent systems (replicas) whose
// steps are far too short to fill the chip one launch at a time: a step of a
// 2000-particle system is a few microseconds of work behind several kernel
// launches.  Here one launch advances a whole batch: workgroup b owns system
// b and runs its n steps with workgroup barriers in place of kernel
// boundaries, reading and writing the system's own device state (the same
// arrays, rotating buffers and counters as db_step).  Every decision and sum
// uses the same device functions as the per-step kernels (fixed-point
// forces, Philox streams keyed by tag, the greedy matching in key order), so
// a batched run is bitwise identical to db_step on each system.
#pragma once

#include "kernels.hpp"

namespace dyb {

// One system of a batch as the kernel sees it (read only).
struct BatchItem {
    Params P;
    Dev D;
};

// Where a system's run stands: read at the start of a launch, written back
// at its end, so consecutive launches of a batch chain on the device alone.
struct BatchState {
    unsigned long long t;    // step of the system
    int cur_x, cur_list;     // current position buffer and cell list
};

constexpr int kBatchMaxThreads = 1024;
// LDS of one batch workgroup: the step tables, a few flags and, in the
// variant that keeps them there, the positions of its system (16 B each).
constexpr uint32_t kBatchLdsTotal = 160u * 1024u;
constexpr uint32_t kBatchLdsStatic = (uint32_t)sizeof(StepTabs) + 256u;

// Workgroup-scope atomic add on global memory: only the owning workgroup
// touches a system's arrays during a batch launch, so the add can complete
// in the local L2 instead of the device-coherent point.
__device__ __forceinline__ uint32_t wg_atomic_add(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_atomic_min64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Device pointers read from a batch item are generic to the compiler (they
// come from memory, not from kernel arguments), and generic accesses compile
// to flat instructions, which also count against the LDS wait counter: a
// wait for an LDS read (the step tables, positions held in LDS) then waits
// for every memory load in flight as well.  The pointers of the hot loops
// pass through the scalar unit and come back typed as global pointers, so
// that the loads through them compile to global loads.
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(__attribute__((address_space(1))) T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void bin_particle_wg(const Params& P, const Dev& D, int lst, uint32_t i, float4 p) {
    const int c = (cell_coord(p.z, P) * (int)P.nc + cell_coord(p.y, P)) * (int)P.nc + cell_coord(p.x, P);
    const uint32_t slot = wg_atomic_add(&D.ccount[lst][c], 1u);
    if (slot < P.cellcap)
        D.cpos[lst][cell_slot(P, (uint32_t)c, slot)] = make_float4(p.x, p.y, p.z, __uint_as_float(i | (type_of(p) << 24)));
    else atomicOr(&D.err[0], kErrOverflow);
}

// Total force on particle i at X (list + bonds), one thread, in 2^-32 fixed
// point.  The loads that need only i (list length, the first 4 list rows,
// the first 2 bond words) are issued together, then the positions they
// name, so that a particle with a short list and few bonds waits for two
// memory round trips; longer lists are taken 8 entries at a time with all
// their loads in flight, further bond slots one by one.
template <bool EXT>
__device__ __forceinline__ Force3 force_site(const Params& P, const StepTabs& T, const Dev& D,
                                             const float4* __restrict__ X, uint32_t i, float4 pi) {
    constexpr int QL = 4, QB = EXT ? 1 : 2;   // (the full variant's extra branches leave room for one bond word)
    const size_t n = P.n;
    const uint32_t ti = type_of(pi);
    const uint32_t nstat = P.stat_max, nslot = P.stat_max + T.cap[ti];
    long long fx = 0, fy = 0, fz = 0;
    const uint32_t* __restrict__ nl = as_global(D.nl);
    const uint32_t* __restrict__ stat = as_global(D.stat);
    const uint32_t* __restrict__ dyn = as_global(D.dyn);
    const uint32_t m = as_global(D.nl_cnt)[i];
    uint32_t nb[QL], bw[QB];
#pragma unroll
    for (int q = 0; q < QL; ++q) nb[q] = (uint32_t)q < P.nlmax ? nl[(size_t)q * n + i] : i;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const uint32_t b = (uint32_t)q;
        bw[q] = b < nslot ? (b < nstat ? stat[(size_t)b * n + i] : dyn[(size_t)(b - nstat) * n + i]) : kEmpty;
    }
    float4 pj[QL], pb[QB];
#pragma unroll
    for (int q = 0; q < QL; ++q) pj[q] = X[(uint32_t)q < m ? nb[q] : i];
#pragma unroll
    for (int q = 0; q < QB; ++q) pb[q] = X[bw[q] != kEmpty ? (bw[q] & kIdxMask) : i];
    // Pairs that need the FP64 evaluation (near the cutoff, across the
    // boundary) are marked and evaluated after the others: a wave then runs
    // as many FP64 evaluations as its busiest lane has, instead of one for
    // every list entry at which any of its lanes needs one.  (Entries from
    // the 33rd on are evaluated at once.)  The sum is exact, so the order
    // does not change the force.
    uint32_t defer = 0u;
#pragma unroll
    for (int q = 0; q < QL; ++q)
        if ((uint32_t)q < m && !pair_force_f32(P, T, D.err, pi, pj[q], ti, fx, fy, fz)) defer |= 1u << q;
    for (uint32_t k0 = QL; k0 < m; k0 += 8) {
        uint32_t nx[8];
        float4 px[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) nx[q] = nl[(size_t)min(k0 + (uint32_t)q, m - 1u) * n + i];
#pragma unroll
        for (int q = 0; q < 8; ++q) px[q] = X[nx[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t k = k0 + (uint32_t)q;
            if (k < m && !pair_force_f32(P, T, D.err, pi, px[q], ti, fx, fy, fz)) {
                if (k < 32u) defer |= 1u << k;
                else pair_force_f64(P, T, D.err, pi, px[q], ti, fx, fy, fz);
            }
        }
    }
    while (defer) {
        const uint32_t k = (uint32_t)__builtin_ctz(defer);
        defer &= defer - 1u;
        const uint32_t j = k >= (uint32_t)QL ? nl[(size_t)k * n + i]
                                             : (k == 0u ? nb[0] : (k == 1u ? nb[1] : (k == 2u ? nb[2] : nb[3])));
        pair_force_f64(P, T, D.err, pi, X[j], ti, fx, fy, fz);
    }
    auto bond = [&](uint32_t b, uint32_t w, float4 pw) {
        const uint32_t j = w & kIdxMask;
        if (b < nstat) bond_force_tab<EXT>(P, T, D, pi, pw, w >> 24, i, j, fx, fy, fz);
        else bond_force_tab<EXT>(P, T, D, pi, pw, T.rbt[(w >> 24) & 0x7Fu], i, j, fx, fy, fz);
    };
#pragma unroll
    for (int q = 0; q < QB; ++q)
        if (bw[q] != kEmpty) bond((uint32_t)q, bw[q], pb[q]);
    for (uint32_t b = QB; b < nslot; ++b) {
        const uint32_t w = b < nstat ? stat[(size_t)b * n + i] : dyn[(size_t)(b - nstat) * n + i];
        if (w != kEmpty) bond(b, w, X[w & kIdxMask]);
    }
    return fix_to_force(D, fx, fy, fz);
}

// Neighbour list of particle i at X from cell list `lst` of the same
// positions (one thread), a z layer of the 27-cell stencil at a time: the
// counts of its 9 cells together, then its entries taken 8 at a time from
// one index space over the 9 cells, with their loads in flight together
// (a cell's entries are not fetched one dependent load after another).
__device__ __forceinline__ void nl_build_site(const Params& P, const StepTabs& T, const Dev& D, int lst,
                                              uint32_t i, float4 pi) {
    const uint32_t* __restrict__ cnt = D.ccount[lst];
    const float4* __restrict__ cp = D.cpos[lst];
    const int nc = (int)P.nc;
    const int cx = cell_coord(pi.x, P), cy = cell_coord(pi.y, P), cz = cell_coord(pi.z, P);
    const float* rrow = T.rl2 + type_of(pi) * kMaxTypes;
    const uint32_t cap = P.cellcap;
    uint32_t m = 0;
    auto consider = [&](float4 q) {
        const uint32_t j = slot_index(q);
        if (j == i) return;
        const float dx = mi_delta_f(pi.x, q.x, P), dy = mi_delta_f(pi.y, q.y, P), dz = mi_delta_f(pi.z, q.z, P);
        if (dx * dx + dy * dy + dz * dz < rrow[slot_type(q)]) {
            if (m < P.nlmax) D.nl[(size_t)m * P.n + i] = j;
            ++m;
        }
    };
#pragma unroll
    for (int g = 0; g < 3; ++g) {                 // z layer oz = g - 1
        uint32_t cell[9], off[10];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int ox = q % 3 - 1, oy = q / 3 - 1;
            cell[q] = (uint32_t)((wrapc(cz + g - 1, nc) * nc + wrapc(cy + oy, nc)) * nc + wrapc(cx + ox, nc));
        }
        uint32_t cn[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) cn[q] = min(cnt[cell[q]], cap);
        off[0] = 0u;
#pragma unroll
        for (int q = 0; q < 9; ++q) off[q + 1] = off[q] + cn[q];
        const uint32_t total = off[9];
        for (uint32_t k0 = 0; k0 < total; k0 += 8) {
            float4 f[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t idx = min(k0 + (uint32_t)e, total - 1u);
                // the cell holding entry idx: the last one whose range starts at or below it
                uint32_t c = cell[0], o = 0u;
#pragma unroll
                for (int q = 1; q < 9; ++q)
                    if (idx >= off[q]) {
                        c = cell[q];
                        o = off[q];
                    }
                f[e] = cp[cell_slot(P, c, idx - o)];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (k0 + (uint32_t)e < total) consider(f[e]);
        }
    }
    if (m > P.nlmax) atomicOr(&D.err[0], kErrNlist);
    D.nl_cnt[i] = m < P.nlmax ? m : P.nlmax;
    D.xref[i] = xref_pack(P, pi);
}

// The same build for the variant that holds the positions in LDS (xs): a
// cell's member slots then carry only the particle index (4 bytes instead of
// a 16-byte position record), and each candidate's position is read from
// LDS, so the build reads a quarter of the bytes from memory.  bin_index_wg
// fills such a list.
__device__ __forceinline__ void bin_index_wg(const Params& P, const Dev& D, int lst, uint32_t i, float4 p) {
    const int c = (cell_coord(p.z, P) * (int)P.nc + cell_coord(p.y, P)) * (int)P.nc + cell_coord(p.x, P);
    const uint32_t slot = wg_atomic_add(as_global(D.ccount[lst]) + c, 1u);
    if (slot < P.cellcap) as_global(reinterpret_cast<uint32_t*>(D.cpos[lst]))[cell_slot(P, (uint32_t)c, slot)] = i;
    else atomicOr(&D.err[0], kErrOverflow);
}

__device__ __forceinline__ void nl_build_site_lds(const Params& P, const StepTabs& T, const Dev& D, int lst,
                                                  uint32_t i, float4 pi, const float4* __restrict__ xs) {
    const uint32_t* __restrict__ cnt = as_global(D.ccount[lst]);
    const uint32_t* __restrict__ ci = as_global(reinterpret_cast<const uint32_t*>(D.cpos[lst]));
    uint32_t* __restrict__ nl = as_global(D.nl);
    const int nc = (int)P.nc;
    const int cx = cell_coord(pi.x, P), cy = cell_coord(pi.y, P), cz = cell_coord(pi.z, P);
    const float* rrow = T.rl2 + type_of(pi) * kMaxTypes;
    const uint32_t cap = P.cellcap;
    uint32_t m = 0;
    auto consider = [&](uint32_t j) {
        if (j == i) return;
        const float4 q = xs[j];
        const float dx = mi_delta_f(pi.x, q.x, P), dy = mi_delta_f(pi.y, q.y, P), dz = mi_delta_f(pi.z, q.z, P);
        if (dx * dx + dy * dy + dz * dz < rrow[type_of(q)]) {
            if (m < P.nlmax) nl[(size_t)m * P.n + i] = j;
            ++m;
        }
    };
#pragma unroll
    for (int g = 0; g < 3; ++g) {                 // z layer oz = g - 1
        uint32_t cell[9], off[10];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int ox = q % 3 - 1, oy = q / 3 - 1;
            cell[q] = (uint32_t)((wrapc(cz + g - 1, nc) * nc + wrapc(cy + oy, nc)) * nc + wrapc(cx + ox, nc));
        }
        uint32_t cn[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) cn[q] = min(cnt[cell[q]], cap);
        off[0] = 0u;
#pragma unroll
        for (int q = 0; q < 9; ++q) off[q + 1] = off[q] + cn[q];
        const uint32_t total = off[9];
        for (uint32_t k0 = 0; k0 < total; k0 += 8) {
            uint32_t e8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t idx = min(k0 + (uint32_t)e, total - 1u);
                uint32_t c = cell[0], o = 0u;
#pragma unroll
                for (int q = 1; q < 9; ++q)
                    if (idx >= off[q]) {
                        c = cell[q];
                        o = off[q];
                    }
                e8[e] = ci[cell_slot(P, c, idx - o)];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (k0 + (uint32_t)e < total) consider(e8[e]);
        }
    }
    if (m > P.nlmax) atomicOr(&D.err[0], kErrNlist);
    as_global(D.nl_cnt)[i] = m < P.nlmax ? m : P.nlmax;
    as_global(D.xref)[i] = xref_pack(P, pi);
}

// n steps of system blockIdx.x.  Per step, as db_step: forces at x_t + BAOAB
// (x_{t+1} is binned and the list rebuilt right after a step that moved
// some particle by more than skin / 2), and the bonding sweep at s = t + 1
// when s is a multiple of the sweep period.  In the sweep, the rounds of the
// greedy matching alternate two key buffers: post keys at both sites of each
// live proposal, claim the proposals that hold the minimum at both sites
// (and try them, Eq. pon), drop the proposals that touch a claimed site.
// Any workgroup size that is a multiple of 64 up to kBatchMaxThreads gives
// the same result: particles are dealt out round robin over the threads and
// every sum is exact.
// With LX the positions of the current step are copied into LDS (dynamic
// LDS of n float4) after every step, and the force, list and sweep passes
// gather neighbour and partner positions from there: a thread walks its
// particles one after another, and each neighbour gather that comes from
// LDS instead of memory shortens that chain by a memory round trip.  Its
// cell lists hold indices only (nl_build_site_lds).  The copy is exact, so
// both variants give the same result.
template <bool EXT, bool LX>
__global__ __launch_bounds__(kBatchMaxThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_batch(const BatchItem* __restrict__ items, BatchState* __restrict__ state, uint32_t nsteps) {
    const BatchItem& B = items[blockIdx.x];
    const Params& P = B.P;
    const Dev& D = B.D;
    const BatchState st0 = state[blockIdx.x];
    const unsigned long long t0 = st0.t;
    __shared__ StepTabs T;
    __shared__ uint32_t flag[3];          // rebuild flags, one per step mod 3
    __shared__ uint32_t more[3];          // live proposals left, one per matching round mod 3
    extern __shared__ float4 xs[];        // with LX: the positions of the current step
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    const uint32_t n = P.n;
    stage_tabs(D, T, tid);
    if (tid < 3) flag[tid] = more[tid] = 0u;
    int xin = st0.cur_x, lcur = st0.cur_list;
    if constexpr (LX) {
        const float4* __restrict__ Xg = D.x[xin];
        for (uint32_t i = tid; i < n; i += bs) xs[i] = Xg[i];
    }
    __syncthreads();
    for (uint32_t k = 0; k < nsteps; ++k) {
        const unsigned long long t = t0 + k, s = t + 1;
        const int lnext = lcur == 2 ? 0 : lcur + 1;
        const bool sweep = P.nrx > 0 && (s % P.period) == 0;
        const int ake = (sweep && P.kt_kinetic) ? 1 : 0;
        if (tid == 0) flag[(k + 1) % 3] = 0u;   // last read two steps ago
        const float4* __restrict__ X;
        if constexpr (LX) X = xs;
        else X = as_global(D.x[xin]);
        const float4* __restrict__ U = as_global(D.u);
        const uint2* __restrict__ XR = as_global(D.xref);
        unsigned long long ke = 0ull;
        for (uint32_t i = tid; i < n; i += bs) {
            const float4 pi = X[i];
            const float4 ui = U[i];
            const uint2 r = XR[i];
            const Force3 F = force_site<EXT>(P, T, D, X, i, pi);
            float4 po;
            ke += advance_particle(P, T, D, xin, i, pi, type_of(pi), F, ui, __float_as_uint(ui.w), s, ake, po);
            if (moved_past_skin(P, r, po)) flag[k % 3] = 1u;
        }
        if (ake) {
            for (int off = 32; off >= 1; off >>= 1) ke += __shfl_xor(ke, off, 64);
            if (__lane_id() == 0 && ke)
                __hip_atomic_fetch_add(&D.ke_fix[ke_slot(P, s)], ke, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        xin ^= 1;
        lcur = lnext;
        const float4* __restrict__ Xn;
        if constexpr (LX) {
            const float4* __restrict__ Xg = D.x[xin];
            for (uint32_t i = tid; i < n; i += bs) xs[i] = Xg[i];
            __syncthreads();
            Xn = xs;
        } else {
            Xn = D.x[xin];
        }
        if (flag[k % 3]) {
            // neighbour lists at x_{t+1}: cell list lcur emptied, filled,
            // then read by the build (steps without a build bin nothing)
            for (uint32_t c = tid; c < P.ncell; c += bs) D.ccount[lcur][c] = 0u;
            if (tid == 0) ++D.rflag[4];       // builds so far, as db_step counts them
            __syncthreads();
            if constexpr (LX) {
                for (uint32_t i = tid; i < n; i += bs) bin_index_wg(P, D, lcur, i, Xn[i]);
                __syncthreads();
                for (uint32_t i = tid; i < n; i += bs) nl_build_site_lds(P, T, D, lcur, i, Xn[i], xs);
            } else {
                for (uint32_t i = tid; i < n; i += bs) bin_particle_wg(P, D, lcur, i, Xn[i]);
                __syncthreads();
                for (uint32_t i = tid; i < n; i += bs) nl_build_site(P, T, D, lcur, i, Xn[i]);
            }
            __syncthreads();
        }
        if (!sweep) continue;
        const float4* __restrict__ Xs = Xn;
        unsigned long long* const B0 = D.best[0];
        unsigned long long* const B1 = D.best[1];
        for (int slot = 0; slot < (int)P.nrx; ++slot) {
            const int a = reaction_at(P.seed, s, (int)P.nrx, slot);
            for (uint32_t i = tid; i < n; i += bs) {
                B0[i] = kNoKey;
                B1[i] = kNoKey;
                D.claimed[i] = 0;
                D.estate[i] = kEdgeNone;
                D.prop[i] = -1;
            }
            if (tid < 3) more[tid] = 0u;
            if (slot == 0 && tid == 0) {      // a new sweep: its event lists start empty
                D.evc[0] = 0u;
                D.evc[1] = 0u;
                D.evc[2] = (uint32_t)s;
                D.evc[3] = (uint32_t)(s >> 32);
            }
            __syncthreads();
            for (uint32_t i = tid; i < n; i += bs) {
                uint32_t tgi = 0;
                const int j = propose_site<1, 4>(P, D, a, Xs, i, 0u, tgi);
                if (j < 0) continue;
                const unsigned long long key = match_key(P, a, s, tgi);
                D.prop[i] = j;
                D.key[i] = key;
                D.estate[i] = kEdgeLive;
                wg_atomic_min64(&B0[i], key);
                wg_atomic_min64(&B0[(uint32_t)j], key);
            }
            uint32_t att = 0, form = 0;
            for (uint32_t r = 0;; ++r) {
                unsigned long long* const Bc = (r & 1u) ? B1 : B0;
                unsigned long long* const Bn = (r & 1u) ? B0 : B1;
                if (tid == 0) more[(r + 1) % 3] = 0u;
                __syncthreads();
                for (uint32_t i = tid; i < n; i += bs) {
                    if (D.estate[i] != kEdgeLive) continue;
                    const uint32_t j = (uint32_t)D.prop[i];
                    const unsigned long long key = D.key[i];
                    if (Bc[i] == key && Bc[j] == key) {
                        D.estate[i] = kEdgeMatched;
                        D.claimed[i] = 1;
                        D.claimed[j] = 1;
                        ++att;
                        form += accept_pair<EXT>(P, D, a, s, Xs, i, j) ? 1u : 0u;
                    }
                }
                __syncthreads();
                for (uint32_t i = tid; i < n; i += bs) {
                    Bc[i] = kNoKey;
                    if (D.estate[i] != kEdgeLive) continue;
                    const uint32_t j = (uint32_t)D.prop[i];
                    if (D.claimed[i] || D.claimed[j]) {
                        D.estate[i] = kEdgeDead;
                    } else {
                        const unsigned long long key = D.key[i];
                        wg_atomic_min64(&Bn[i], key);
                        wg_atomic_min64(&Bn[j], key);
                        more[r % 3] = 1u;
                    }
                }
                __syncthreads();
                if (!more[r % 3]) break;
            }
            count_add(D, a, kCtrAttempt, att);
            count_add(D, a, kCtrForm, form);
            uint32_t broke = 0;
            for (uint32_t i = tid; i < n; i += bs) broke += break_site<EXT>(P, D, a, s, i, Xs);
            count_add(D, a, kCtrBreak, broke);
            __syncthreads();
        }
        if (tid == 0) D.ke_fix[ke_slot(P, s) ^ 1u] = 0ull;   // the next sweep's slot, as db_step leaves it
    }
    // hand the state back in the form db_step leaves it: step slots, no list
    // rebuild pending, the cell list of db_step's next build empty, round-1
    // key buffer clear
    for (uint32_t i = tid; i < n; i += bs) D.best[1][i] = kNoKey;
    __syncthreads();
    {
        uint32_t* __restrict__ cl = D.ccount[D.rflag[3]];
        for (uint32_t c = tid; c < P.ncell; c += bs) cl[c] = 0u;
    }
    if (tid == 0) {
        D.stepv[0] = D.stepv[1] = t0 + nsteps;
        D.rflag[0] = D.rflag[1] = D.rflag[2] = 0u;
        BatchState st;
        st.t = t0 + nsteps;
        st.cur_x = xin;
        st.cur_list = lcur;
        state[blockIdx.x] = st;
    }
}

// Spatial renumbering of system blockIdx.x inside one workgroup, launched
// before every chunk of batched steps: what the periodic sort of db_step
// does over the whole chip.  New indices in (cell, type) order from the
// current cell list (each thread takes a contiguous run of buckets), every
// per-particle array permuted with bond partners remapped, the current cell
// list binned again under the new indices and the neighbour lists rebuilt.
// Nothing computed depends on the numbering (tags key every decision, sums
// are exact), so a batched run stays equal to db_step; the sweep's per-site
// scratch is reset at every sweep and the other position buffer is written
// before it is read, so neither is permuted.
__global__ __launch_bounds__(kBatchMaxThreads)
void k_batch_sort(const BatchItem* __restrict__ items, const BatchState* __restrict__ state) {
    const BatchItem& B = items[blockIdx.x];
    const Params& P = B.P;
    const Dev& D = B.D;
    const BatchState st = state[blockIdx.x];
    const int xin = st.cur_x, lst = st.cur_list;
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    const size_t n = P.n;
    __shared__ StepTabs T;
    stage_tabs(D, T, tid);
    // the current positions binned into cell list `lst`, the other two empty
    // (db_step keeps its cell lists in its own way)
    for (int l = 0; l < 3; ++l)
        for (uint32_t c = tid; c < P.ncell; c += bs) D.ccount[l][c] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += bs) bin_particle_wg(P, D, lst, i, D.x[xin][i]);
    __syncthreads();
    const uint32_t nbk = P.ncell * P.ntypes;
    const uint32_t per = (nbk + bs - 1) / bs;
    const uint32_t b0 = min(tid * per, nbk), b1 = min(b0 + per, nbk);
    uint32_t cnt = 0;
    for (uint32_t b = b0; b < b1; ++b) cnt += bucket_count(P, D, lst, b);
    uint32_t total;
    uint32_t at = block_exclusive_scan(cnt, &total);
    for (uint32_t b = b0; b < b1; ++b) {
        uint32_t c, t;
        bucket_cell_type(P, D, b, c, t);
        uint32_t m = D.ccount[lst][c];
        m = m < P.cellcap ? m : P.cellcap;
        const float4* cp = D.cpos[lst];
        for (uint32_t k = 0; k < m; ++k) {
            const float4 q = cp[cell_slot(P, c, k)];
            if (slot_type(q) == t) D.newidx[slot_index(q)] = at++;
        }
    }
    __syncthreads();
    float4* __restrict__ X = D.x[xin];
    for (uint32_t i = tid; i < n; i += bs) {
        const uint32_t j = D.newidx[i];
        if (j >= n) continue;              // only after a cell overflow, already reported
        D.x_alt[j] = X[i];
        D.u_alt[j] = D.u[i];
        D.img_alt[j] = D.img[i];
        D.img_alt[n + j] = D.img[n + i];
        D.img_alt[2 * n + j] = D.img[2 * n + i];
        const uint32_t tg = D.tag[i];
        D.tag_alt[j] = tg;
        D.rtag[tg] = j;
        D.occ_alt[j] = D.occ[i];
        D.mol_alt[j] = D.mol[i];
        for (uint32_t k = 0; k < P.cap_max; ++k) D.dyn_alt[k * n + j] = remap_slot(D, D.dyn[k * n + i]);
        for (uint32_t k = 0; k < P.stat_max; ++k) D.stat_alt[k * n + j] = remap_slot(D, D.stat[k * n + i]);
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += bs) {
        X[i] = D.x_alt[i];
        D.u[i] = D.u_alt[i];
        D.img[i] = D.img_alt[i];
        D.img[n + i] = D.img_alt[n + i];
        D.img[2 * n + i] = D.img_alt[2 * n + i];
        D.tag[i] = D.tag_alt[i];
        D.occ[i] = D.occ_alt[i];
        D.mol[i] = D.mol_alt[i];
        for (uint32_t k = 0; k < P.cap_max; ++k) D.dyn[k * n + i] = D.dyn_alt[k * n + i];
        for (uint32_t k = 0; k < P.stat_max; ++k) D.stat[k * n + i] = D.stat_alt[k * n + i];
    }
    for (uint32_t c = tid; c < P.ncell; c += bs) D.ccount[lst][c] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += bs) bin_particle_wg(P, D, lst, i, X[i]);
    __syncthreads();
    for (uint32_t i = tid; i < n; i += bs) nl_build_site(P, T, D, lst, i, X[i]);
}

}  // namespace dyb
