// HIP kernels of the dynamic-bonding Langevin MD step (gfx950, wave64).
//
// Step structure (three launches per time step, plus the sweep every n
// steps):
//
//   k_step      forces at x_t (neighbour list, WCA on every listed pair,
//               static and dynamic bonds), closing half kick of the previous
//               step, then B-A-O-A of BAOAB, wrap, and the test whether some
//               particle has moved more than half the skin since the last
//               list build.  Forces are accumulated in 64-bit fixed point, so
//               the sum does not depend on the order in which neighbours are
//               visited.
//   k_binr      only after a step that set that flag: x_{t+1} binned into a
//   k_nlist     cell list, then the neighbour lists rebuilt from it (both
//               return at once otherwise).
//   sweep       per reaction (order redrawn every sweep, Sec. 2.3):
//               k_propose -> (k_claim, k_kill)* -> k_finish -> k_break.
//               The matching reproduces the sequential greedy matching in
//               ascending priority key exactly: a proposal is claimed as soon
//               as its key is the minimum over all live proposals touching
//               either of its sites (local-minimum rounds); the last rounds run
//               inside one workgroup.  Acceptance (Eq. pon) is evaluated by the
//               thread that claims the pair and writes both sites' slots.
#pragma once

#include "device.hpp"

namespace dyb {

// ------------------------------------------------------------ force kernel
struct Force3 { float x, y, z; };

// Slot of the kinetic-energy sum that the sweep with step key s reads: sweeps
// alternate between two slots, so the last kernel of a sweep can clear the
// slot of the next one while its own is still being read.
__device__ __forceinline__ uint32_t ke_slot(const Params& P, unsigned long long s) {
    return (uint32_t)((s / P.period) & 1ull);
}

// Temperature of the sweep with step key s: the set point, or the kinetic
// temperature sum m v^2 / (3 N) accumulated by the step before it.
__device__ __forceinline__ double sweep_kT(const Params& P, const Dev& D, unsigned long long s) {
    return P.kt_kinetic ? (double)D.ke_fix[ke_slot(P, s)] * kFixInv / (3.0 * (double)P.n) : P.kT;
}

// Tether bond: U = U_att + U_rep with U_att = k e^{1/(l_c0 - r)} / (l_max - r)
// for r > l_c0 and U_rep = k e^{1/(r - l_c1)} / (r - l_min) for r < l_c1,
// zero in between; returns U, dU/dr in du.
__device__ __forceinline__ double tether_u(double r, double k, double lmin, double lc1, double lc0, double lmax,
                                           double* du) {
#pragma clang fp contract(off)
    double U = 0.0, d = 0.0;
    if (r > lc0) {
        const double e = exp_det(1.0 / (lc0 - r));
        U += k * e / (lmax - r);
        d += k * e * (1.0 / ((lc0 - r) * (lc0 - r) * (lmax - r)) + 1.0 / ((lmax - r) * (lmax - r)));
    }
    if (r < lc1) {
        const double e = exp_det(1.0 / (r - lc1));
        U += k * e / (r - lmin);
        d -= k * e * (1.0 / ((r - lc1) * (r - lc1) * (r - lmin)) + 1.0 / ((r - lmin) * (r - lmin)));
    }
    *du = d;
    return U;
}

// Energy U_b(r) of bond type bt (the acceptance and slip factors of the
// sweep use it): harmonic k/2 (r - r0)^2, FENE -k R0^2/2 ln(1 - r^2/R0^2),
// tether as above.  The reaction window keeps r inside the bond's range.
__device__ __forceinline__ double bond_energy(const Params& P, uint32_t bt, double r) {
#pragma clang fp contract(off)
    const uint32_t kind = P.bkind[bt];
    if (kind == 0u) {
        const double d = r - P.br0[bt];
        return (0.5 * P.bk[bt]) * (d * d);
    }
    if (kind == 1u) {
        const double x2 = (r * r) / P.bR02[bt];
        return -0.5 * P.bk[bt] * P.br0[bt] * P.br0[bt] * log1p_det(-x2);
    }
    double du;
    return tether_u(r, P.bk[bt], P.blmin[bt], P.blc1[bt], P.blc0[bt], P.blmax[bt], &du);
}

// Melting modifier: P = P_init (1 - g) + P_melt g with
// g = [tanh(lambda (T - T_melt)) + 1] / 2.
__device__ __forceinline__ double melt_mix(double p_init, double p_melt, double lam, double tm, double T) {
#pragma clang fp contract(off)
    const double g = 0.5 * (tanh_det(lam * (T - tm)) + 1.0);
    return p_init * (1.0 - g) + p_melt * g;
}

// Slip bond: P_off = P0_off exp(a sqrt(U_b / kT)), at most 1; at kT = 0 the
// factor is 1 for U_b = 0 and unbounded otherwise.
__device__ __forceinline__ double slip_prob(double p0, double a, double U, double kT) {
#pragma clang fp contract(off)
    if (kT > 0.0) {
        const double q = p0 * exp_det(a * sqrt(U / kT));
        return q < 1.0 ? q : 1.0;
    }
    return (U > 0.0 && a > 0.0) ? 1.0 : p0;
}

// Report a bond outside its range (FENE r >= R0, tether outside (l_min, l_max)).
__device__ __forceinline__ void bond_range_error(const Dev& D, uint32_t i, uint32_t j) {
    if (atomicOr(&D.err[0], kErrFene) == 0u) {
        D.err[1] = D.tag[i];
        D.err[2] = D.tag[j];
    }
}

// Bond force on site i from partner position pj (bond type bt), in FP64 from
// the exact minimum-image separation.
__device__ __forceinline__ void bond_force(const Params& P, const Dev& D, float4 pi, float4 pj,
                                           uint32_t bt, uint32_t i, uint32_t j,
                                           long long& fx, long long& fy, long long& fz,
                                           double* e) {
#pragma clang fp contract(off)
    const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
    const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
    const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    double f;
    if (P.bkind[bt] == 1u) {                      // FENE: F_i = k / (1 - r^2/R0^2) d
        const double g = 1.0 - r2 * P.binvR02[bt];
        if (!(g > 0.0)) {
            bond_range_error(D, i, j);
            return;
        }
        f = P.bk[bt] * rcp64(g);
        if (e) *e += 0.5 * (-0.5 * P.bk[bt] * P.bR02[bt] * log(g));
    } else if (P.bkind[bt] == 2u) {               // tether: F_i = (dU/dr) / r d
        const double r = sqrt(r2);
        if (!(r > P.blmin[bt] && r < P.blmax[bt])) {
            bond_range_error(D, i, j);
            return;
        }
        double du;
        const double U = tether_u(r, P.bk[bt], P.blmin[bt], P.blc1[bt], P.blc0[bt], P.blmax[bt], &du);
        f = du / r;
        if (e) *e += 0.5 * U;
    } else {                                      // harmonic: F_i = k (r - r0) / r d
        if (!(r2 > 0.0)) return;
        const double ir = rsqrt64(r2);
        const double dr = r2 * ir - P.br0[bt];
        f = P.bk[bt] * dr * ir;
        if (e) *e += 0.5 * (0.5 * P.bk[bt] * dr * dr);
    }
    fx += to_fix(f * dx, D.err);
    fy += to_fix(f * dy, D.err);
    fz += to_fix(f * dz, D.err);
}

// WCA force on pi from the cell-slot entry pj (position + index/type bits).
// Screened in FP32 with a safety margin; pairs that survive are evaluated in
// FP64.  The cutoff test r < 2^(1/6) sigma_ij is the oracle's: away from the
// cutoff it is decided on r^2, within 1e-14 of it on the correctly rounded r.
__device__ __forceinline__ void pair_force(const Params& P, const Dev& D, float4 pi, float4 pj, uint32_t ti,
                                           long long& fx, long long& fy, long long& fz, double* e) {
#pragma clang fp contract(off)
    const int pt = (int)ti * kMaxTypes + (int)slot_type(pj);
    const float fdx = mi_delta_f(pi.x, pj.x, P);
    const float fdy = mi_delta_f(pi.y, pj.y, P);
    const float fdz = mi_delta_f(pi.z, pj.z, P);
    if (fdx * fdx + fdy * fdy + fdz * fdz >= P.rc2_pre[pt]) return;
    const PairTab& pp = D.pair[pt];
    const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
    const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
    const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
    double r2;
    {
#pragma clang fp contract(off)
        r2 = (dx * dx + dy * dy) + dz * dz;
    }
    if (r2 >= pp.rc2_hi) return;
    if (r2 > pp.rc2_lo && !(sqrt(r2) < pp.rc)) return;
    // F_i = -24 eps (sigma/r)^6 (2 (sigma/r)^6 - 1) / r^2 * d
    const double ir2 = rcp64(r2);
    const double sr2 = pp.sig2 * ir2;
    const double sr6 = sr2 * sr2 * sr2;
    const double f = pp.eps24 * sr6 * (2.0 * sr6 - 1.0) * ir2;
    fx -= to_fix(f * dx, D.err);
    fy -= to_fix(f * dy, D.err);
    fz -= to_fix(f * dz, D.err);
    if (e) *e += 0.5 * (4.0 * pp.eps * (sr6 * sr6 - sr6) + pp.eps);
}

// WCA force on pi from a position-array entry pj (type in the w bits).
__device__ __forceinline__ void pair_force_xt(const Params& P, const Dev& D, float4 pi, float4 pj, uint32_t ti,
                                              long long& fx, long long& fy, long long& fz, double* e) {
    const float4 q = make_float4(pj.x, pj.y, pj.z, __uint_as_float(type_of(pj) << 24));
    pair_force(P, D, pi, q, ti, fx, fy, fz, e);
}

// WCA force on pi from neighbour-list entry pj (type in the w bits).  When no
// component of x_j - x_i needs a periodic image, the FP32 difference is the
// correctly rounded separation, and pairs inside 0.98 rc (where
// 2 (sigma/r)^6 - 1 > 0.12, no cancellation) are evaluated in FP32.  Pairs
// near the cutoff and pairs across the boundary take the FP64 path of
// pair_force.
__device__ __forceinline__ void pair_force_list(const Params& P, const Dev& D, float4 pi, float4 pj, uint32_t ti,
                                                long long& fx, long long& fy, long long& fz) {
    const int pt = (int)ti * kMaxTypes + (int)type_of(pj);
    const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    if (fabsf(dx) <= P.halfLf && fabsf(dy) <= P.halfLf && fabsf(dz) <= P.halfLf) {
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= P.rc2_pre[pt]) return;
        if (r2 < P.rc2_in[pt]) {
            const float ir2 = __builtin_amdgcn_rcpf(r2);
            const float sr2 = P.sig2f[pt] * ir2;
            const float sr6 = sr2 * sr2 * sr2;
            const float f = P.eps24f[pt] * sr6 * (2.0f * sr6 - 1.0f) * ir2;
            fx -= to_fix((double)(f * dx), D.err);
            fy -= to_fix((double)(f * dy), D.err);
            fz -= to_fix((double)(f * dz), D.err);
            return;
        }
    }
    const float4 q = make_float4(pj.x, pj.y, pj.z, __uint_as_float(type_of(pj) << 24));
    pair_force(P, D, pi, q, ti, fx, fy, fz, nullptr);
}

// Static and dynamic bond forces on particle i.
__device__ __forceinline__ void bond_forces(const Params& P, const Dev& D, const float4* __restrict__ X,
                                            uint32_t i, float4 pi, uint32_t ti,
                                            long long& fx, long long& fy, long long& fz, double* e) {
    for (uint32_t s = 0; s < P.stat_max; ++s) {
        const uint32_t w = D.stat[(size_t)s * P.n + i];
        if (w == kEmpty) break;
        const uint32_t j = w & kIdxMask;
        bond_force(P, D, pi, X[j], w >> 24, i, j, fx, fy, fz, e);
    }
    const uint32_t cap = P.cap[ti];
    for (uint32_t s = 0; s < cap; ++s) {
        const uint32_t w = D.dyn[(size_t)s * P.n + i];
        if (w == kEmpty) continue;
        const uint32_t j = w & kIdxMask;
        bond_force(P, D, pi, X[j], P.rbt[(w >> 24) & 0x7Fu], i, j, fx, fy, fz, e);
    }
}

__device__ __forceinline__ Force3 fix_to_force(const Dev& D, long long fx, long long fy, long long fz) {
    return Force3{(float)((double)fx * kFixInv), (float)((double)fy * kFixInv),
                  (float)((double)fz * kFixInv)};
}

// Total force on particle i at positions X from its neighbour list (valid
// for X: every pair within the interaction range is listed until some
// particle has moved by skin / 2 since the build, and the step that moves it
// that far rebuilds the lists); optional per-particle energy (half of each
// pair and bond energy).  Candidates are screened in FP32 with a safety
// margin; pairs that survive are evaluated in FP64 with the same cutoff test
// as the oracle (r < 2^(1/6) sigma_ij).  Each contribution is rounded to
// 2^-32 and summed in 64-bit integers.
__device__ __forceinline__ Force3 force_on(const Params& P, const Dev& D, const float4* __restrict__ X,
                                           uint32_t i, float4 pi, uint32_t ti, double* e) {
    long long fx = 0, fy = 0, fz = 0;
    const uint32_t m = D.nl_cnt[i];
    for (uint32_t k = 0; k < m; ++k) pair_force_xt(P, D, pi, X[D.nl[(size_t)k * P.n + i]], ti, fx, fy, fz, e);
    bond_forces(P, D, X, i, pi, ti, fx, fy, fz, e);
    return fix_to_force(D, fx, fy, fz);
}

__global__ void k_clear_counts(const Params P, const Dev D, int lst) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell; c += gridDim.x * blockDim.x)
        D.ccount[lst][c] = 0u;
}

// Insert one wave's particles (lanes with `valid`) into cell list `lst`,
// with one counter atomic per run of consecutive lanes in the same cell:
// particles are numbered in cell order, so a wave's 64 lanes fall into a
// few such runs, and same-address atomics are taken one at a time.  Each
// lane's slot is the run's base plus its place in the run.  All 64 lanes
// must call this together.
__device__ __forceinline__ void bin_wave(const Params& P, const Dev& D, int lst, uint32_t i, bool valid,
                                         float4 p) {
    const int c = valid ? (cell_coord(p.z, P) * (int)P.nc + cell_coord(p.y, P)) * (int)P.nc + cell_coord(p.x, P)
                        : -1;
    const uint32_t lane = __lane_id();
    const int cprev = __shfl_up(c, 1u, 64);
    const bool head = lane == 0u || c != cprev;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = (2ull << lane) - 1ull;         // lanes 0..lane (all for lane 63)
    const uint32_t h = 63u - (uint32_t)__clzll((long long)(heads & upto));   // this lane's run head
    const unsigned long long above = heads & ~upto;
    const uint32_t next = above ? (uint32_t)__ffsll((long long)above) - 1u : 64u;
    uint32_t base = 0;
    if (head && valid) base = atomicAdd(&D.ccount[lst][c], next - lane);
    base = __shfl(base, (int)h, 64);
    if (valid) {
        const uint32_t slot = base + (lane - h);
        if (slot < P.cellcap)
            D.cpos[lst][cell_slot(P, (uint32_t)c, slot)] = make_float4(p.x, p.y, p.z, __uint_as_float(i | (type_of(p) << 24)));
        else atomicOr(&D.err[0], kErrOverflow);
    }
}

__global__ void k_bin(const Params P, const Dev D, int xin, int lst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < P.n;
    bin_wave(P, D, lst, i, valid, valid ? D.x[xin][i] : make_float4(0.f, 0.f, 0.f, 0.f));
}

// Cell lists: lists 0 and 1 take turns holding the positions of the latest
// neighbour-list build; rflag[3] names the one the next build bins into, which
// is kept empty (the build clears the other one, and the step after a build
// switches rflag[3] over).  List 2 serves the spatial renumbering.
constexpr int kSortList = 2;

// Binning for a neighbour-list build: does nothing unless the rebuild flag
// `f3` is set (by the step that moved some particle by more than skin / 2,
// or by a renumbering); then inserts every particle at X into cell list
// rflag[3].  Steps that need no build pay only this launch, not the binning.
__global__ void k_binr(const Params P, const Dev D, int xin, int f3) {
    if (D.rflag[f3] == 0u) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < P.n;
    bin_wave(P, D, (int)D.rflag[3], i, valid, valid ? D.x[xin][i] : make_float4(0.f, 0.f, 0.f, 0.f));
}

// Forces (and per-particle energies) at the current positions into f4[off + i].
__global__ void k_eval(const Params P, const Dev D, int xin, uint32_t off) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const float4 pi = D.x[xin][i];
    double e = 0.0;
    const Force3 f = force_on(P, D, D.x[xin], i, pi, type_of(pi), &e);
    D.f4[off + i] = make_float4(f.x, f.y, f.z, (float)e);
}

// u = v - h F / m (turn full-step velocities into the stored form).
__global__ void k_init_u(const Params P, const Dev D, int xin, uint32_t off) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const float hm = P.h * P.inv_mass[type_of(D.x[xin][i])];
    const float4 f = D.f4[off + i];
    float4 u = D.u[i];
    u.x -= hm * f.x;
    u.y -= hm * f.y;
    u.z -= hm * f.z;
    D.u[i] = u;
}

// After a frozen sweep changed the bonds: keep v = u + h F/m unchanged.
__global__ void k_fix_u(const Params P, const Dev D, int xin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const float hm = P.h * P.inv_mass[type_of(D.x[xin][i])];
    const float4 fo = D.f4[i];
    const float4 fn = D.f4[P.n + i];
    float4 u = D.u[i];
    u.x += hm * fo.x - hm * fn.x;
    u.y += hm * fo.y - hm * fn.y;
    u.z += hm * fo.z - hm * fn.z;
    D.u[i] = u;
}

// sum m v^2 of the full-step velocities (v = u + h F/m, F in f4) into ke_fix.
__global__ __launch_bounds__(256) void k_ke_accum(const Params P, const Dev D, int xin, unsigned long long s) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ke = 0ull;
    if (i < P.n) {
        const uint32_t ti = type_of(D.x[xin][i]);
        const float hm = P.h * P.inv_mass[ti];
        const float4 u = D.u[i], f = D.f4[i];
        const float vx = u.x + hm * f.x, vy = u.y + hm * f.y, vz = u.z + hm * f.z;
        const double v2 = ((double)vx * vx + (double)vy * vy) + (double)vz * vz;
        ke = (unsigned long long)rint((double)P.mass[ti] * v2 * 4294967296.0);
    }
    for (int off = 32; off >= 1; off >>= 1) ke += __shfl_xor(ke, off, 64);
    if (__lane_id() == 0 && ke) atomicAdd(&D.ke_fix[ke_slot(P, s)], ke);
}

// Block-wide exclusive scan (blockDim a multiple of 64, at most 1024).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[16];
    const uint32_t lane = __lane_id(), wid = threadIdx.x / 64;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    const uint32_t nw = blockDim.x / 64;
    for (uint32_t w = 0; w < nw; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// Rest of one BAOAB step for particle i once its force F at x_t is known:
// closing half kick of step t-1 (B), opening half kick (B), half drift (A),
// Ornstein-Uhlenbeck velocity update with Philox Gaussians (O), half drift
// (A), wrap into [-L/2, L/2), then write x_{t+1} (returned in po) and u
// (with the particle's tag in its w word, where the next step reads it).
// Returns m v^2 in 2^-32 fixed point when accum_ke is set.
template <class Tabs>
__device__ __forceinline__ unsigned long long advance_particle(const Params& P, const Tabs& T, const Dev& D, int xin,
                                                               uint32_t i, float4 pi, uint32_t ti,
                                                               Force3 F, float4 u, uint32_t tag,
                                                               unsigned long long s, int accum_ke, float4& po) {
    // The order of every rounding is written out (explicit fmaf, no implicit
    // contraction), so that the step gives the same bits in every kernel that
    // inlines it.
#pragma clang fp contract(off)
    const float hm = T.hm[ti];
    float vx = fmaf(hm, F.x, u.x), vy = fmaf(hm, F.y, u.y), vz = fmaf(hm, F.z, u.z);
    vx = fmaf(hm, F.x, vx);
    vy = fmaf(hm, F.y, vy);
    vz = fmaf(hm, F.z, vz);
    float x = fmaf(P.h, vx, pi.x), y = fmaf(P.h, vy, pi.y), z = fmaf(P.h, vz, pi.z);
    const Word4 w = philox((uint32_t)s, (uint32_t)(s >> 32), tag, 0u, P.seed, stream_k1(kThermo, 0, 0));
    // Box-Muller: u1 in (0, 1], u2 in [0, 1)
    const float u1a = ((float)w.w0 + 1.0f) * 0x1.0p-32f;
    const float u1b = ((float)w.w2 + 1.0f) * 0x1.0p-32f;
    const float ra = sqrtf(-2.0f * __logf(u1a));
    const float rb = sqrtf(-2.0f * __logf(u1b));
    const float ta = 6.28318530717958647692f * ((float)w.w1 * 0x1.0p-32f);
    const float sa = __sinf(ta), ca = __cosf(ta);
    const float cb = __cosf(6.28318530717958647692f * ((float)w.w3 * 0x1.0p-32f));
    const float sd = T.noise_sd[ti];
    vx = fmaf(P.c1, vx, sd * (ra * ca));
    vy = fmaf(P.c1, vy, sd * (ra * sa));
    vz = fmaf(P.c1, vz, sd * (rb * cb));
    x = fmaf(P.h, vx, x);
    y = fmaf(P.h, vy, y);
    z = fmaf(P.h, vz, z);
    int ix = 0, iy = 0, iz = 0;
    if (x < -P.halfLf) { x += P.Lf; --ix; }
    if (x >= P.halfLf) { x -= P.Lf; ++ix; }
    if (y < -P.halfLf) { y += P.Lf; --iy; }
    if (y >= P.halfLf) { y -= P.Lf; ++iy; }
    if (z < -P.halfLf) { z += P.Lf; --iz; }
    if (z >= P.halfLf) { z -= P.Lf; ++iz; }
    if (ix | iy | iz) {
        D.img[i] += ix;
        D.img[P.n + i] += iy;
        D.img[2 * P.n + i] += iz;
    }
    po = make_float4(x, y, z, __uint_as_float(ti));
    D.x[xin ^ 1][i] = po;
    D.u[i] = make_float4(vx, vy, vz, __uint_as_float(tag));   // the tag rides in the w word
    if (!accum_ke) return 0ull;
    const double v2 = ((double)vx * vx + (double)vy * vy) + (double)vz * vz;
    return (unsigned long long)rint((double)T.mass[ti] * v2 * 4294967296.0);
}

constexpr int kTileThreads = 512;
// The tables of one tile fit 32 KB of LDS, so that four 512-thread
// workgroups share a CU (twice the tables, 1728 halo cells and 2048 entries,
// allowed two and made the 200k gel's step 2 % slower).
constexpr int kTileMaxHalo = 1000;      // halo cells of one tile, (t+2)^3 <= 1000 (t <= 8)
constexpr int kTileMaxEntries = 1024;   // particles staged in LDS per tile
constexpr int kTileChunk = (kTileMaxHalo + kTileThreads - 1) / kTileThreads;   // halo cells per thread in the scan
constexpr int kTileLoads = kTileMaxEntries / kTileThreads;                     // staged entries per thread
constexpr int kTileMaxCore = 512;       // core particles whose stencil rows are dealt out as work items

// Workgroups are dealt round-robin to the 8 XCDs.  This remaps the workgroup
// id so that each XCD gets a contiguous run of work items (particles are kept
// in cell order, so a run is a compact slab of space whose data fits that
// XCD's L2).
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t per = nb / 8u, rem = nb % 8u, xcd = b % 8u;
    return xcd * per + (xcd < rem ? xcd : rem) + b / 8u;
}

// Append j to the neighbour list of i when it lies within the list radius of
// their type pair (only pairs that interact or can react are listed).
__device__ __forceinline__ void nl_consider(const Params& P, const Dev& D, const float* rl2, uint32_t i, float4 pi,
                                            float4 pj, uint32_t& m) {
    const float dx = mi_delta_f(pi.x, pj.x, P), dy = mi_delta_f(pi.y, pj.y, P), dz = mi_delta_f(pi.z, pj.z, P);
    if (dx * dx + dy * dy + dz * dz < rl2[slot_type(pi) * kMaxTypes + slot_type(pj)]) {
        if (m < P.nlmax) D.nl[(size_t)m * P.n + i] = slot_index(pj);
        ++m;
    }
}

// Neighbour lists: for every particle, the indices of all particles closer
// than r_list = r_search + skin at the current positions; a list stays
// complete for pairs within r_search until some particle has moved by
// skin / 2 from where it was built.  Built from the cell list `lst` of those
// positions, one workgroup per tile of cells: the cell counts of the tile and
// its one-cell halo are scanned in LDS, the halo's particles (position +
// index/type words) are staged in LDS (each thread issues its loads together,
// locating its entries' cells by binary search over the scanned offsets),
// and the stencils of the core particles are scanned as work items of one
// particle and one row of 3 cells (9 per particle, each a contiguous LDS
// range) dealt out round robin over the threads.  Tiles with more than
// kTileMaxCore core particles visit each particle's 27 cells in one thread,
// and tiles whose halo holds more than kTileMaxEntries particles read the
// same stencil from global memory.
// Does nothing unless the rebuild flag `f3` (set by k_step when a particle
// has moved by more than skin / 2, or by a renumbering) is set; the grid is
// a few hundred workgroups, so that the launch is cheap when nothing moved
// that far.  Reads cell list rflag[3] (filled by k_binr) and empties the
// core cells of the other one, which the next build fills.  Compiled for 8
// waves per SIMD (four workgroups per CU; at 57 VGPRs only three fit): the
// build's phases are latency-bound, and the fourth workgroup cut its time by
// 11 % at 4 M and 16 M particles.
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_nlist(const Params P, const Dev D, int f3) {
    if (D.rflag[f3] == 0u) return;
    const int lst = (int)D.rflag[3];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&D.rflag[4], 1u);   // builds so far
    __shared__ float rl2[kMaxTypes * kMaxTypes];   // list radii, indexed by lane-varying type pairs
    __shared__ float4 ent[kTileMaxEntries];
    __shared__ uint32_t hoff[kTileMaxHalo + 1];
    __shared__ uint32_t hglob[kTileMaxHalo];       // global cell index of each halo cell
    __shared__ uint16_t ecell[kTileMaxEntries];    // halo cell of each staged entry
    __shared__ uint16_t core[kTileMaxEntries];     // staged entries that lie in the tile core
    __shared__ uint8_t hshift[kTileMaxHalo];       // periodic image of each halo cell (2 bits per axis)
    __shared__ uint32_t pcnt[kTileMaxCore];        // neighbours found so far
    __shared__ uint16_t prow0[kTileMaxCore];       // first halo row of its 3 x 3 x 3 stencil
    __shared__ uint32_t ncore;
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = xcd_block();
    const int nc = (int)P.nc;
    const int bx = (int)(tile % P.ntile[0]), by = (int)((tile / P.ntile[0]) % P.ntile[1]);
    const int bz = (int)(tile / (P.ntile[0] * P.ntile[1]));
    const int x0 = bx * (int)P.tile[0], y0 = by * (int)P.tile[1], z0 = bz * (int)P.tile[2];
    const int ex = min((int)P.tile[0], nc - x0), ey = min((int)P.tile[1], nc - y0), ez = min((int)P.tile[2], nc - z0);
    const int hx = ex + 2, hy = ey + 2, hz = ez + 2, nh = hx * hy * hz;
    // halo cell h = (iz * hy + iy) * hx + ix; quotients of these small
    // integers (< 2^11) are taken in FP32 and corrected, not with the
    // integer division sequence
    const float rx = 1.0f / (float)hx, rxy = 1.0f / (float)(hx * hy);
    auto qdiv = [](int a, int b, float rb) {
        int q = (int)((float)a * rb);
        q += (q + 1) * b <= a ? 1 : 0;
        q -= q * b > a ? 1 : 0;
        return q;
    };
    auto split = [&](int h, int& ix, int& iy, int& iz) {
        iz = qdiv(h, hx * hy, rxy);
        const int r = h - iz * hx * hy;
        iy = qdiv(r, hx, rx);
        ix = r - iy * hx;
    };
    auto hcell = [&](int h) {
        int ix, iy, iz;
        split(h, ix, iy, iz);
        return (wrapc(z0 - 1 + iz, nc) * nc + wrapc(y0 - 1 + iy, nc)) * nc + wrapc(x0 - 1 + ix, nc);
    };
    // 1: the halo cell lies below cell 0 along that axis (its particles are
    // shifted by -L), 2: above cell nc - 1 (+L); staged positions then form
    // one continuous frame and plain differences are minimum images
    auto hcode = [&](int h) {
        int ix, iy, iz;
        split(h, ix, iy, iz);
        auto c1 = [&](int g) { return g < 0 ? 1u : (g >= nc ? 2u : 0u); };
        return c1(x0 - 1 + ix) | (c1(y0 - 1 + iy) << 2) | (c1(z0 - 1 + iz) << 4);
    };
    auto is_core = [&](int h) {
        int ix, iy, iz;
        split(h, ix, iy, iz);
        return ix >= 1 && ix <= ex && iy >= 1 && iy <= ey && iz >= 1 && iz <= ez;
    };
    const uint32_t* __restrict__ cnt = D.ccount[lst];
    const float4* __restrict__ cp = D.cpos[lst];
    if (tid < kMaxTypes * kMaxTypes) rl2[tid] = P.rl2[tid];
    if (tid == 0) ncore = 0;
    // halo counts -> exclusive offsets (each thread scans a contiguous chunk)
    // (loads issued unconditionally from clamped cells, then masked, so that
    // they are all in flight together)
    const int chunk = (nh + kTileThreads - 1) / kTileThreads;
    uint32_t loc[kTileChunk], gc[kTileChunk];
#pragma unroll
    for (int q = 0; q < kTileChunk; ++q) {
        gc[q] = (uint32_t)hcell(min((int)tid * chunk + q, nh - 1));
        loc[q] = cnt[gc[q]];
    }
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kTileChunk; ++q) {
        const int h = (int)tid * chunk + q;
        const uint32_t c = (q < chunk && h < nh) ? (loc[q] < P.cellcap ? loc[q] : P.cellcap) : 0u;
        loc[q] = c;
        sum += c;
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, &total);
#pragma unroll
    for (int q = 0; q < kTileChunk; ++q) {
        const int h = (int)tid * chunk + q;
        if (q < chunk && h < nh) {
            hoff[h] = run;
            hglob[h] = gc[q];
            hshift[h] = (uint8_t)hcode(h);
        }
        run += loc[q];
    }
    if (tid == 0) hoff[nh] = total;
    __syncthreads();
    bool over = false;
    if (total == 0u) {
        // nothing in this tile or its halo
    } else if (total <= (uint32_t)kTileMaxEntries) {
        // stage entry e: its cell h is the last one with hoff[h] <= e; loads
        // from clamped entries are issued together, stores masked after
        int hv[kTileLoads];
        float4 v[kTileLoads];
#pragma unroll
        for (int q = 0; q < kTileLoads; ++q) {
            const uint32_t e = min(tid + (uint32_t)q * kTileThreads, total - 1u);
            int lo = 0;                       // hoff[0] = 0 <= e < hoff[nh]
            static_assert(kTileMaxHalo <= 1024, "binary search over at most 1024 halo cells");
#pragma unroll
            for (int step = 512; step >= 1; step >>= 1)
                if (lo + step < nh && hoff[lo + step] <= e) lo += step;
            hv[q] = lo;
            v[q] = cp[cell_slot(P, hglob[lo], e - hoff[lo])];
        }
        // threads past the end rewrite the last entry with its own value, so
        // the stores need no branch (which would pull the loads after it)
        auto shifted = [&](float x, uint32_t code) {
            return code == 1u ? x - P.Lf : (code == 2u ? x + P.Lf : x);
        };
#pragma unroll
        for (int q = 0; q < kTileLoads; ++q) {
            const uint32_t e = min(tid + (uint32_t)q * kTileThreads, total - 1u);
            const uint32_t code = hshift[hv[q]];
            float4 w = v[q];
            w.x = shifted(w.x, code & 3u);
            w.y = shifted(w.y, (code >> 2) & 3u);
            w.z = shifted(w.z, code >> 4);
            ent[e] = w;
            ecell[e] = (uint16_t)hv[q];
        }
#pragma unroll
        for (int q = 0; q < kTileLoads; ++q)
            if (tid + (uint32_t)q * kTileThreads >= total) hv[q] = -1;
        // core entries: wave ballot, one LDS atomic per wave
#pragma unroll
        for (int q = 0; q < kTileLoads; ++q) {
            const uint32_t e = tid + (uint32_t)q * kTileThreads;
            const bool c = hv[q] >= 0 && is_core(hv[q]);
            const unsigned long long mask = __ballot(c);
            if (mask) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const int leader = __ffsll((long long)mask) - 1;
                uint32_t base = 0;
                if (__lane_id() == leader) base = atomicAdd(&ncore, (uint32_t)__popcll(mask));
                base = __shfl(base, leader, 64);
                if (c) core[base + rank] = (uint16_t)e;
            }
        }
        __syncthreads();
        if (ncore <= (uint32_t)kTileMaxCore) {
            // work items: (core particle, stencil row), 9 rows of 3 cells per
            // particle, each a contiguous range of staged entries; items are
            // dealt out round robin
            for (uint32_t p = tid; p < ncore; p += kTileThreads) {
                int ix, iy, iz;
                split(ecell[core[p]], ix, iy, iz);
                prow0[p] = (uint16_t)(((iz - 1) * hy + (iy - 1)) * hx + (ix - 1));
                pcnt[p] = 0u;
            }
            __syncthreads();
            for (uint32_t it = tid; it < 9u * ncore; it += kTileThreads) {
                const uint32_t p = it / 9u, r = it - 9u * p;
                const uint32_t ep = core[p];
                const float4 pi = ent[ep];
                const uint32_t hr = prow0[p] + ((r / 3u) * (uint32_t)hy + (r % 3u)) * (uint32_t)hx;
                const uint32_t lo = hoff[hr], hi = hoff[hr + 3];
                const float* rrow = rl2 + slot_type(pi) * kMaxTypes;
                for (uint32_t e2 = lo; e2 < hi; ++e2) {
                    if (e2 == ep) continue;
                    const float4 q = ent[e2];
                    const float dx = q.x - pi.x, dy = q.y - pi.y, dz = q.z - pi.z;
                    if (dx * dx + dy * dy + dz * dz < rrow[slot_type(q)]) {
                        const uint32_t k = atomicAdd(&pcnt[p], 1u);
                        if (k < P.nlmax) D.nl[(size_t)k * P.n + slot_index(pi)] = slot_index(q);
                    }
                }
            }
            __syncthreads();
            for (uint32_t q = tid; q < ncore; q += kTileThreads) {
                const float4 pi = ent[core[q]];
                const uint32_t m = pcnt[q];
                over |= m > P.nlmax;
                D.nl_cnt[slot_index(pi)] = m < P.nlmax ? m : P.nlmax;
                D.xref[slot_index(pi)] = xref_pack(P, pi);
            }
        } else {
            for (uint32_t q = tid; q < ncore; q += kTileThreads) {
                const uint32_t e = core[q];
                const int h = ecell[e];
                const float4 pi = ent[e];
                const uint32_t i = slot_index(pi);
                const float* rrow = rl2 + slot_type(pi) * kMaxTypes;
                int ix, iy, iz;
                split(h, ix, iy, iz);
                uint32_t m = 0;
                for (int oz = -1; oz <= 1; ++oz) {
                    for (int oy = -1; oy <= 1; ++oy) {
                        const int hr = ((iz + oz) * hy + (iy + oy)) * hx + (ix - 1);
                        const uint32_t lo = hoff[hr], hi = hoff[hr + 3];
                        for (uint32_t e2 = lo; e2 < hi; ++e2) {
                            if (e2 == e) continue;
                            const float4 q2 = ent[e2];
                            const float dx = q2.x - pi.x, dy = q2.y - pi.y, dz = q2.z - pi.z;
                            if (dx * dx + dy * dy + dz * dz < rrow[slot_type(q2)]) {
                                if (m < P.nlmax) D.nl[(size_t)m * P.n + i] = slot_index(q2);
                                ++m;
                            }
                        }
                    }
                }
                over |= m > P.nlmax;
                D.nl_cnt[i] = m < P.nlmax ? m : P.nlmax;
                D.xref[i] = xref_pack(P, pi);
            }
        }
    } else {
        for (int h = (int)tid; h < nh; h += kTileThreads) {
            if (!is_core(h)) continue;
            const uint32_t o = hoff[h], m0 = hoff[h + 1] - o;
            const uint32_t hc = (uint32_t)hcell(h);
            for (uint32_t k0 = 0; k0 < m0; ++k0) {
                const float4 pi = cp[cell_slot(P, hc, k0)];
                const uint32_t i = slot_index(pi);
                const int cx = cell_coord(pi.x, P), cy = cell_coord(pi.y, P), cz = cell_coord(pi.z, P);
                uint32_t m = 0;
                for (int oz = -1; oz <= 1; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int c = (wrapc(cz + oz, nc) * nc + wrapc(cy + oy, nc)) * nc + wrapc(cx + ox, nc);
                            uint32_t mc = cnt[c];
                            mc = mc < P.cellcap ? mc : P.cellcap;
                            for (uint32_t kk = 0; kk < mc; ++kk) {
                                const float4 pj = cp[cell_slot(P, (uint32_t)c, kk)];
                                if (slot_index(pj) != i) nl_consider(P, D, rl2, i, pi, pj, m);
                            }
                        }
                over |= m > P.nlmax;
                D.nl_cnt[i] = m < P.nlmax ? m : P.nlmax;
                D.xref[i] = xref_pack(P, pi);
            }
        }
    }
    if (over) atomicOr(&D.err[0], kErrNlist);
    // the other list's cells of this tile's core, for the next build
    uint32_t* __restrict__ nxt = D.ccount[lst ^ 1];
    for (int q = (int)tid; q < ex * ey * ez; q += kTileThreads) {
        const int cz = q / (ex * ey), r = q - cz * ex * ey, cy = r / ex, cx = r - cy * ex;
        nxt[((z0 + cz) * nc + (y0 + cy)) * nc + (x0 + cx)] = 0u;
    }
}

// Copy the step tables (built on the host at commit, kept in device memory)
// into LDS, 16 bytes per thread.
__device__ __forceinline__ void stage_tabs(const Dev& D, StepTabs& T, uint32_t tid) {
    const uint4* __restrict__ src = reinterpret_cast<const uint4*>(D.tabs);
    uint4* dst = reinterpret_cast<uint4*>(&T);
    for (uint32_t k = tid; k < sizeof(StepTabs) / 16; k += blockDim.x) dst[k] = src[k];
}

// WCA force on pi from neighbour pj (type in the w bits), constants from LDS.
// When no component of x_j - x_i needs a periodic image, the FP32 difference
// is the correctly rounded separation, and pairs inside 0.98 rc (where
// 2 (sigma/r)^6 - 1 > 0.12, no cancellation) are evaluated in FP32.  Pairs
// near the cutoff and pairs across the boundary are screened in FP32 and
// evaluated in FP64 with the oracle's cutoff test r < 2^(1/6) sigma_ij.
// pair_force_f32 takes the screen and the FP32 evaluation and returns false
// for a pair that still needs pair_force_f64; pair_force_tab runs both.
__device__ __forceinline__ bool pair_force_f32(const Params& P, const StepTabs& T, uint32_t* err, float4 pi,
                                               float4 pj, uint32_t ti, long long& fx, long long& fy,
                                               long long& fz) {
#pragma clang fp contract(off)
    const int pt = (int)ti * kMaxTypes + (int)type_of(pj);
    const float rc2p = T.rc2_pre[pt];
    float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    if (fabsf(dx) <= P.halfLf && fabsf(dy) <= P.halfLf && fabsf(dz) <= P.halfLf) {
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (r2 >= rc2p) return true;
        if (r2 < T.rc2_in[pt]) {
            const float ir2 = __builtin_amdgcn_rcpf(r2);
            const float sr2 = T.sig2f[pt] * ir2;
            const float sr6 = sr2 * sr2 * sr2;
            const float f = T.eps24f[pt] * sr6 * (2.0f * sr6 - 1.0f) * ir2;
            fx -= to_fix((double)(f * dx), err);
            fy -= to_fix((double)(f * dy), err);
            fz -= to_fix((double)(f * dz), err);
            return true;
        }
    } else {
        dx = mi_delta_f(pi.x, pj.x, P);
        dy = mi_delta_f(pi.y, pj.y, P);
        dz = mi_delta_f(pi.z, pj.z, P);
        if (fmaf(dz, dz, fmaf(dy, dy, dx * dx)) >= rc2p) return true;
    }
    return false;
}

__device__ __forceinline__ void pair_force_f64(const Params& P, const StepTabs& T, uint32_t* err, float4 pi,
                                               float4 pj, uint32_t ti, long long& fx, long long& fy,
                                               long long& fz) {
#pragma clang fp contract(off)
    const PairTab& pp = T.pair[(int)ti * kMaxTypes + (int)type_of(pj)];
    const double ex = mi_delta(pi.x, pj.x, P.L, P.invL);
    const double ey = mi_delta(pi.y, pj.y, P.L, P.invL);
    const double ez = mi_delta(pi.z, pj.z, P.L, P.invL);
    double r2;
    {
#pragma clang fp contract(off)
        r2 = (ex * ex + ey * ey) + ez * ez;
    }
    if (r2 >= pp.rc2_hi) return;
    if (r2 > pp.rc2_lo && !(sqrt(r2) < pp.rc)) return;
    const double ir2 = rcp64(r2);
    const double sr2 = pp.sig2 * ir2;
    const double sr6 = sr2 * sr2 * sr2;
    const double f = pp.eps24 * sr6 * (2.0 * sr6 - 1.0) * ir2;
    fx -= to_fix(f * ex, err);
    fy -= to_fix(f * ey, err);
    fz -= to_fix(f * ez, err);
}

__device__ __forceinline__ void pair_force_tab(const Params& P, const StepTabs& T, uint32_t* err, float4 pi,
                                               float4 pj, uint32_t ti, long long& fx, long long& fy,
                                               long long& fz) {
    if (!pair_force_f32(P, T, err, pi, pj, ti, fx, fy, fz)) pair_force_f64(P, T, err, pi, pj, ti, fx, fy, fz);
}

// Bond force on site i from partner j (bond type bt), FP64 from the exact
// minimum-image separation, constants from LDS.
// EXT: the system has tether bonds or rate modifiers (kernels are built in
// two variants, so that systems without them keep the lean register budget).
template <bool EXT>
__device__ __forceinline__ void bond_force_tab(const Params& P, const StepTabs& T, const Dev& D, float4 pi,
                                               float4 pj, uint32_t bt, uint32_t i, uint32_t j,
                                               long long& fx, long long& fy, long long& fz) {
#pragma clang fp contract(off)
    const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
    const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
    const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    double f;
    if (T.bkind[bt] == 1u) {                      // FENE: F_i = k / (1 - r^2/R0^2) d
        const double g = 1.0 - r2 * T.binvR02[bt];
        if (!(g > 0.0)) {
            bond_range_error(D, i, j);
            return;
        }
        f = T.bk[bt] * rcp64(g);
    } else if (EXT && T.bkind[bt] == 2u) {        // tether: F_i = (dU/dr) / r d
        const double r = sqrt(r2);
        if (!(r > T.blmin[bt] && r < T.blmax[bt])) {
            bond_range_error(D, i, j);
            return;
        }
        double du;
        (void)tether_u(r, T.bk[bt], T.blmin[bt], T.blc1[bt], T.blc0[bt], T.blmax[bt], &du);
        f = du / r;
    } else {                                      // harmonic: F_i = k (r - r0) / r d
        if (!(r2 > 0.0)) return;
        const double ir = rsqrt64(r2);
        f = T.bk[bt] * (r2 * ir - T.br0[bt]) * ir;
    }
    fx += to_fix(f * dx, D.err);
    fy += to_fix(f * dy, D.err);
    fz += to_fix(f * dz, D.err);
}

// One BAOAB step t -> s = t + 1 over 256 / TPP particles per workgroup.
//
// Force phase: TPP threads share a particle; each takes every TPP-th entry
// of the particle's neighbour list and every TPP-th bond slot (static slots,
// then dynamic ones).  All loads that depend only on the particle index (its
// position, list length, the first Q list entries per thread, the bond
// words) are issued together, then the neighbour and partner positions
// together, so that a thread waits for about three memory round trips
// instead of two per neighbour.  Each contribution is rounded to 2^-32 and
// the partial sums are added into LDS as 64-bit integers (exact, so the
// split and the order do not change the result).
//
// Integration phase: the first 256 / TPP threads (whole waves) integrate the
// workgroup's particles, one per thread (advance_particle), and test the
// list: a particle farther than skin / 2 from where its list was built sets
// the flag of step t+1, read by the k_binr and k_nlist launched right after
// (which bin x_{t+1} and rebuild the lists only then).  The other waves have
// retired by then, so no lane idles through the integration.
//   xin = buffer of x_t, sp = t mod 2, f3 = t mod 3.
//   QB (if not 0) = list entries per thread issued up front.
// Thread 0 also retires the rebuild flag of step t (consumed by the k_nlist
// of step t - 1), switching the cell list of the next build when it was set.
__device__ __forceinline__ void retire_rebuild_flag(const Dev& D, int f3) {
    if (D.rflag[f3]) {
        D.rflag[3] ^= 1u;
        D.rflag[f3] = 0u;
    }
}

template <int TPP, int QB = 0, bool EXT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_step(const Params P, const Dev D, int xin, int sp,
                                              int f3, int accum_ke) {
    static_assert(TPP >= 1 && TPP <= 64, "256 threads per workgroup");
    constexpr int PPB = 256 / TPP;                       // particles per workgroup
    constexpr uint32_t kIntThreads = PPB > 64 ? PPB : 64;   // whole waves that integrate
    constexpr int Q = QB ? QB : (4 / TPP > 1 ? 4 / TPP : 1);   // list entries per thread issued up front
    constexpr int QX = 8 / TPP > 1 ? 8 / TPP : 1;              // further entries per thread, issued with the gathers
    constexpr int BQ = 8 / TPP > 1 ? 8 / TPP : 1;       // bond slots per thread issued up front
    __shared__ StepTabs T;
    __shared__ unsigned long long fsum[3][PPB];
    const uint32_t tid = threadIdx.x;
    const uint32_t base = xcd_block() * PPB;
    const uint32_t i = base + tid / TPP, lane = tid % TPP;
    const uint32_t gtid = blockIdx.x * blockDim.x + tid;
    const size_t n = P.n;
    const float4* __restrict__ X = D.x[xin];
    const uint32_t nslot = P.stat_max + P.cap_max;
    // loads that need only i
    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t m = 0;
    uint32_t nb[Q], bw[BQ];
#pragma unroll
    for (int q = 0; q < Q; ++q) nb[q] = 0u;
#pragma unroll
    for (int q = 0; q < BQ; ++q) bw[q] = kEmpty;
    if (i < P.n) {
        pi = X[i];
        m = D.nl_cnt[i];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t k = lane + (uint32_t)q * TPP;
            if (k < P.nlmax) nb[q] = D.nl[k * n + i];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const uint32_t b = lane + (uint32_t)q * TPP;
            if (b < P.stat_max) bw[q] = D.stat[b * n + i];
            else if (b < nslot) bw[q] = D.dyn[(b - P.stat_max) * n + i];
        }
    }
    stage_tabs(D, T, tid);
    if (tid < PPB) fsum[0][tid] = fsum[1][tid] = fsum[2][tid] = 0ull;
    const unsigned long long s = D.stepv[sp] + 1ull;
    if (gtid == 0) {
        D.stepv[sp ^ 1] = s;
        retire_rebuild_flag(D, f3);
    }
    __syncthreads();
    if (i < P.n) {
        const uint32_t ti = type_of(pi);
        // neighbour and partner positions
        float4 pj[Q], pb[BQ];
        // (unconditional loads from clamped indices, so that all are in flight
        // together; entries past the list and empty slots are masked below)
#pragma unroll
        for (int q = 0; q < Q; ++q) pj[q] = X[lane + (uint32_t)q * TPP < m ? nb[q] : i];
#pragma unroll
        for (int q = 0; q < BQ; ++q) pb[q] = X[bw[q] != kEmpty ? (bw[q] & kIdxMask) : i];
        // list rows past the first Q per thread, only where the list has them
        uint32_t nx[QX];
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const uint32_t k = lane + (uint32_t)(Q + q) * TPP;
            nx[q] = k < m ? D.nl[k * n + i] : i;
        }
        long long fx = 0, fy = 0, fz = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t k = lane + (uint32_t)q * TPP;
            if (k < m) pair_force_tab(P, T, D.err, pi, pj[q], ti, fx, fy, fz);
        }
        // longer lists (a few particles per wave): their next entries were
        // loaded together with the first gathers, their positions now
        if (m > (uint32_t)(Q * TPP)) {
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const uint32_t k = lane + (uint32_t)(Q + q) * TPP;
                if (k < m) pair_force_tab(P, T, D.err, pi, X[nx[q]], ti, fx, fy, fz);
            }
            for (uint32_t k = lane + (uint32_t)(Q + QX) * TPP; k < m; k += TPP)
                pair_force_tab(P, T, D.err, pi, X[D.nl[k * n + i]], ti, fx, fy, fz);
        }
        auto bond = [&](uint32_t b, uint32_t w, float4 pw) {
            const uint32_t j = w & kIdxMask;
            if (b < P.stat_max) bond_force_tab<EXT>(P, T, D, pi, pw, w >> 24, i, j, fx, fy, fz);
            else if (b - P.stat_max < T.cap[ti])
                bond_force_tab<EXT>(P, T, D, pi, pw, T.rbt[(w >> 24) & 0x7Fu], i, j, fx, fy, fz);
        };
#pragma unroll
        for (int q = 0; q < BQ; ++q)
            if (bw[q] != kEmpty) bond(lane + (uint32_t)q * TPP, bw[q], pb[q]);
        for (uint32_t b = lane + (uint32_t)BQ * TPP; b < nslot; b += TPP) {
            const uint32_t w = b < P.stat_max ? D.stat[b * n + i] : D.dyn[(b - P.stat_max) * n + i];
            if (w != kEmpty) bond(b, w, X[w & kIdxMask]);
        }
        atomicAdd(&fsum[0][tid / TPP], (unsigned long long)fx);
        atomicAdd(&fsum[1][tid / TPP], (unsigned long long)fy);
        atomicAdd(&fsum[2][tid / TPP], (unsigned long long)fz);
    }
    // the integrating wave fetches its particles' state before the barrier
    const uint32_t i2 = base + tid;
    const bool own = tid < (uint32_t)PPB && i2 < P.n;
    float4 p2 = make_float4(0.f, 0.f, 0.f, 0.f), u2 = p2;
    uint2 r2 = make_uint2(0u, 0u);
    if (own) {
        p2 = X[i2];
        u2 = D.u[i2];
        r2 = D.xref[i2];
    }
    __syncthreads();
    if (tid >= kIntThreads) return;
    unsigned long long ke = 0ull;
    if (own) {
        const uint32_t t2 = type_of(p2);
        const Force3 F = fix_to_force(D, (long long)fsum[0][tid], (long long)fsum[1][tid], (long long)fsum[2][tid]);
        float4 po;
        ke = advance_particle(P, T, D, xin, i2, p2, t2, F, u2, __float_as_uint(u2.w), s, accum_ke, po);
        if (moved_past_skin(P, r2, po)) D.rflag[f3 == 2 ? 0 : f3 + 1] = 1u;
    }
    if (accum_ke) {
        for (int off = 32; off >= 1; off >>= 1) ke += __shfl_xor(ke, off, 64);
        if (__lane_id() == 0 && ke) atomicAdd(&D.ke_fix[ke_slot(P, s)], ke);
    }
}

// One BAOAB step t -> s = t + 1 with one thread per particle (the default
// for large systems): the thread issues its particle's loads (position,
// velocity, list position, tag, list length, the first 4 list entries and 2
// bond words) together, then the 4 neighbour and 2 partner positions
// together, takes further list entries 4 at a time the same way and further
// bond slots one by one, and goes on to the integration with its force in
// registers (no LDS reduction, one barrier).  Same arguments and the same
// result bit for bit as k_step<TPP>.  Compiled for 6 waves per SIMD (78
// VGPRs, no spill): with 4 bond words up front it took 88 VGPRs and ran 5,
// 4 % slower at 4 M and 16 M particles; 8 waves spill.
template <bool EXT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_step1(const Params P, const Dev D, int xin, int sp,
                                                                                       int f3, int accum_ke) {
    constexpr int Q = 4, BQ = 2;
    __shared__ StepTabs T;
    const uint32_t tid = threadIdx.x;
    const uint32_t i = xcd_block() * 256u + tid;
    const uint32_t gtid = blockIdx.x * blockDim.x + tid;
    const size_t n = P.n;
    const float4* __restrict__ X = D.x[xin];
    const uint32_t nslot = P.stat_max + P.cap_max;
    const bool live = i < P.n;
    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f), ui = pi;
    uint2 ri = make_uint2(0u, 0u);
    uint32_t m = 0;
    uint32_t nb[Q], bw[BQ];
#pragma unroll
    for (int q = 0; q < Q; ++q) nb[q] = 0u;
#pragma unroll
    for (int q = 0; q < BQ; ++q) bw[q] = kEmpty;
    if (live) {
        pi = X[i];
        ui = D.u[i];
        ri = D.xref[i];
        m = D.nl_cnt[i];
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if ((uint32_t)q < P.nlmax) nb[q] = D.nl[(size_t)q * n + i];
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const uint32_t b = (uint32_t)q;
            if (b < P.stat_max) bw[q] = D.stat[b * n + i];
            else if (b < nslot) bw[q] = D.dyn[(b - P.stat_max) * n + i];
        }
    }
    stage_tabs(D, T, tid);
    const unsigned long long s = D.stepv[sp] + 1ull;
    if (gtid == 0) {
        D.stepv[sp ^ 1] = s;
        retire_rebuild_flag(D, f3);
    }
    __syncthreads();
    unsigned long long ke = 0ull;
    if (live) {
        const uint32_t ti = type_of(pi);
        float4 pj[Q], pb[BQ];
#pragma unroll
        for (int q = 0; q < Q; ++q) pj[q] = X[(uint32_t)q < m ? nb[q] : i];
#pragma unroll
        for (int q = 0; q < BQ; ++q) pb[q] = X[bw[q] != kEmpty ? (bw[q] & kIdxMask) : i];
        long long fx = 0, fy = 0, fz = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if ((uint32_t)q < m) pair_force_tab(P, T, D.err, pi, pj[q], ti, fx, fy, fz);
        for (uint32_t k0 = Q; k0 < m; k0 += Q) {
#pragma unroll
            for (int q = 0; q < Q; ++q) nb[q] = D.nl[(size_t)min(k0 + (uint32_t)q, m - 1u) * n + i];
#pragma unroll
            for (int q = 0; q < Q; ++q) pj[q] = X[nb[q]];
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (k0 + (uint32_t)q < m) pair_force_tab(P, T, D.err, pi, pj[q], ti, fx, fy, fz);
        }
        auto bond = [&](uint32_t b, uint32_t w, float4 pw) {
            const uint32_t j = w & kIdxMask;
            if (b < P.stat_max) bond_force_tab<EXT>(P, T, D, pi, pw, w >> 24, i, j, fx, fy, fz);
            else if (b - P.stat_max < T.cap[ti])
                bond_force_tab<EXT>(P, T, D, pi, pw, T.rbt[(w >> 24) & 0x7Fu], i, j, fx, fy, fz);
        };
#pragma unroll
        for (int q = 0; q < BQ; ++q)
            if (bw[q] != kEmpty) bond((uint32_t)q, bw[q], pb[q]);
        for (uint32_t b = BQ; b < nslot; ++b) {
            const uint32_t w = b < P.stat_max ? D.stat[b * n + i] : D.dyn[(b - P.stat_max) * n + i];
            if (w != kEmpty) bond(b, w, X[w & kIdxMask]);
        }
        const Force3 F = fix_to_force(D, fx, fy, fz);
        float4 po;
        ke = advance_particle(P, T, D, xin, i, pi, ti, F, ui, __float_as_uint(ui.w), s, accum_ke, po);
        if (moved_past_skin(P, ri, po)) D.rflag[f3 == 2 ? 0 : f3 + 1] = 1u;
    }
    if (accum_ke) {
        for (int off = 32; off >= 1; off >>= 1) ke += __shfl_xor(ke, off, 64);
        if (__lane_id() == 0 && ke) atomicAdd(&D.ke_fix[ke_slot(P, s)], ke);
    }
}

// ------------------------------------------------------------ spatial sort
// Particles are renumbered in cell order (slot order inside a cell) so that
// the particles of a tile and their bond partners sit close together in
// memory.  Nothing computed depends on the numbering: random streams and
// tie-breaks use tags, sums are in fixed point.
// Cells are visited in Morton (Z-curve) order of their coordinates (table
// D.corder, built at commit): any run of consecutive particles then fills a
// compact block of space, so the neighbours a workgroup gathers, and the run
// of workgroups one XCD takes, stay within few cache lines and one L2.
// Buckets are (cell, type) in cell-major order: a cell's particles stay
// together whatever their types, so bonded partners (of other types) and
// neighbours sit next to each other in memory.  (Type-major order, every
// type in a block of its own, made the step 3 % slower at 200k particles and
// 6 % at 4 M: a particle's partners then lie in another block.)
__device__ __forceinline__ void bucket_cell_type(const Params& P, const Dev& D, uint32_t b, uint32_t& c,
                                                 uint32_t& t) {
    const uint32_t r = b / P.ntypes;
    t = b - r * P.ntypes;
    c = D.corder[r];
}

__device__ __forceinline__ uint32_t bucket_count(const Params& P, const Dev& D, int lst, uint32_t b) {
    uint32_t c, t;
    bucket_cell_type(P, D, b, c, t);
    uint32_t m = D.ccount[lst][c];
    m = m < P.cellcap ? m : P.cellcap;
    const float4* cp = D.cpos[lst];
    uint32_t r = 0;
    for (uint32_t k = 0; k < m; ++k) r += slot_type(cp[cell_slot(P, c, k)]) == t;
    return r;
}

__global__ __launch_bounds__(256) void k_cell_scan_blocks(const Params P, const Dev D, int lst) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nbk = P.ntypes * P.ncell;
    const uint32_t m = b < nbk ? bucket_count(P, D, lst, b) : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(m, &tot);
    if (b < nbk) D.cstart[b] = ex;
    if (threadIdx.x == 0) D.cbsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_sort_assign(const Params P, const Dev D, int lst) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= P.ntypes * P.ncell) return;
    uint32_t c, t;
    bucket_cell_type(P, D, b, c, t);
    uint32_t m = D.ccount[lst][c];
    m = m < P.cellcap ? m : P.cellcap;
    uint32_t at = D.cstart[b] + D.cbsum[blockIdx.x];
    const float4* cp = D.cpos[lst];
    for (uint32_t k = 0; k < m; ++k) {
        const float4 q = cp[cell_slot(P, c, k)];
        if (slot_type(q) == t) D.newidx[slot_index(q)] = at++;
    }
}

__device__ __forceinline__ uint32_t remap_slot(const Dev& D, uint32_t w) {
    return w == kEmpty ? kEmpty : (D.newidx[w & kIdxMask] | (w & ~kIdxMask));
}

__global__ __launch_bounds__(256) void k_sort_scatter(const Params P, const Dev D, int xin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const uint32_t j = D.newidx[i];
    if (j >= P.n) return;                  // only after a cell overflow, already reported
    const size_t n = P.n;
    D.x_alt[j] = D.x[xin][i];
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

__global__ __launch_bounds__(256) void k_sort_copyback(const Params P, const Dev D, int xin, int f3) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {                    // indices changed: rebuild the neighbour lists now
        retire_rebuild_flag(D, f3);  // (a build that just ran leaves the other cell list empty)
        D.rflag[f3] = 1u;
    }
    if (i >= P.n) return;
    const size_t n = P.n;
    D.x[xin][i] = D.x_alt[i];
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

// ------------------------------------------------------------ sweep kernels
__device__ __forceinline__ int sweep_reaction(const Params& P, unsigned long long s, int slot) {
    __shared__ int alpha;
    if (threadIdx.x == 0) alpha = reaction_at(P.seed, s, (int)P.nrx, slot);
    __syncthreads();
    return alpha;
}

// Matching priority of a proposal by site i (tag tgi): first Philox word of
// the MATCH stream in the high half, the tag in the low half (unique keys).
__device__ __forceinline__ unsigned long long match_key(const Params& P, int a, unsigned long long s, uint32_t tgi) {
    const Word4 w = philox((uint32_t)s, (uint32_t)(s >> 32), tgi, 0u, P.seed, stream_k1(kMatch, a, 0));
    return ((unsigned long long)w.w0 << 32) | tgi;
}

// Proposal of site i for reaction a (Sec. 2.3, Fig. sweep a): TPP threads
// share the site (`lane` = this thread's rank in the group); each scans every
// TPP-th neighbour-list entry and the group keeps the lexicographic minimum of
// (|r - r0|, tag).  Sites that cannot propose leave after loading their
// position and occupancy.  For a proposer, the loads that need only i (the
// first Q list entries per thread, the bond words) are issued together, then
// everything the candidates need (position, occupancy, molecule, tag), so
// that it waits for about four memory round trips.  The group issues 4 list
// entries up front (TPP when TPP > 4): lists hold a few entries (1.7 on
// average in the gel), and every entry issued is a separate row of the
// slot-major list, a cache line or more for the group's sites, which at
// millions of sites is most of the kernel's traffic.  Returns the chosen
// partner (the same on every thread of the group) or -1; `tgi` receives the
// site's tag.
template <int TPP, int Q = (TPP < 4 ? 4 / TPP : 1)>
__device__ __forceinline__ int propose_site(const Params& P, const Dev& D, int a, const float4* __restrict__ X,
                                            uint32_t i, uint32_t lane, uint32_t& tgi_out) {
    const size_t n = P.n;
    // sites that cannot propose (wrong type, full valence) leave after one load
    const float4 pi = X[i];
    const uint32_t occ_i = D.occ[i];
    const uint32_t ti = type_of(pi);
    const uint32_t ta = P.ra[a], tb = P.rb[a];
    if (ti != ta && ti != tb) return -1;
    if (occ_i >= P.cap[ti]) return -1;
    const uint32_t m = D.nl_cnt[i];
    uint32_t nb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t k = lane + (uint32_t)q * TPP;
        nb[q] = k < P.nlmax ? D.nl[k * n + i] : 0u;
    }
    // partners already bonded to i (any bond) are excluded; slots beyond the
    // site's valence are empty
    uint32_t mine[kMaxValence + kMaxStatic];
#pragma unroll
    for (int k = 0; k < kMaxValence; ++k)
        mine[k] = (uint32_t)k < P.cap_max ? (D.dyn[(size_t)k * n + i] & kIdxMask) : kIdxMask;
#pragma unroll
    for (int k = 0; k < kMaxStatic; ++k)
        mine[kMaxValence + k] = (uint32_t)k < P.stat_max ? (D.stat[(size_t)k * n + i] & kIdxMask) : kIdxMask;
    const bool avoid = P.rself[a] != 0u;
    const uint32_t mol_i = avoid ? D.mol[i] : 0u;
    const uint32_t tgi = D.tag[i];
    const uint32_t want = ti == ta ? tb : ta;
    const uint32_t cap_want = P.cap[want];
    const double rmin = P.rmin[a], rmax = P.rmax[a], r0 = P.r0[a];
    const float rmax2 = P.rmax2_pre[a], rmin2 = P.rmin2_pre[a];
    // the best candidate so far; its tag is read only when an exact tie of
    // |r - r0| needs it (kTagUnread until then), so that a candidate costs a
    // position and an occupancy gather (and its molecule only when the
    // reaction avoids its own molecule)
    constexpr uint32_t kTagUnread = 0xFFFFFFFFu;   // tags are below 2^24
    double best_score = 0.0;
    uint32_t best_tag = kTagUnread;
    int best_j = -1;
    // candidate j: partner type, free, not yet bonded to i, other molecule if
    // required, inside [r_min, r_max] (FP32 screen, then the exact FP64 r);
    // keep the smallest (|r - r0|, tag)
    auto consider = [&](uint32_t j, float4 pj, uint32_t occ_j, uint32_t mol_j) {
        if (type_of(pj) != want) return;
        if (occ_j >= cap_want) return;
        bool bonded = false;
#pragma unroll
        for (int q = 0; q < kMaxValence + kMaxStatic; ++q) bonded |= mine[q] == j;
        if (bonded) return;
        if (avoid && mol_j == mol_i) return;
        const float fdx = mi_delta_f(pi.x, pj.x, P);
        const float fdy = mi_delta_f(pi.y, pj.y, P);
        const float fdz = mi_delta_f(pi.z, pj.z, P);
        const float fr2 = fdx * fdx + fdy * fdy + fdz * fdz;
        if (fr2 > rmax2 || fr2 < rmin2) return;
        const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
        const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
        const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
        const double r = norm3(dx, dy, dz);
        if (!(r >= rmin && r <= rmax)) return;
        const double score = fabs(r - r0);
        if (best_j < 0 || score < best_score) {
            best_score = score;
            best_tag = kTagUnread;
            best_j = (int)j;
        } else if (score == best_score) {           // exact tie: the smaller tag wins
            if (best_tag == kTagUnread) best_tag = D.tag[best_j];
            const uint32_t tgj = D.tag[j];
            if (tgj < best_tag) {
                best_tag = tgj;
                best_j = (int)j;
            }
        }
    };
    // the neighbour list (rebuilt right after every step that needed it) holds
    // every pair within r_search >= r_max
    float4 pj[Q];
    uint32_t oj[Q], mj[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t j = lane + (uint32_t)q * TPP < m ? nb[q] : i;
        pj[q] = X[j];
        oj[q] = D.occ[j];
        mj[q] = avoid ? D.mol[j] : 0u;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (lane + (uint32_t)q * TPP < m) consider(nb[q], pj[q], oj[q], mj[q]);
    for (uint32_t k = lane + (uint32_t)Q * TPP; k < m; k += TPP) {
        const uint32_t j = D.nl[k * n + i];
        consider(j, X[j], D.occ[j], avoid ? D.mol[j] : 0u);
    }
#pragma unroll
    for (int o = TPP / 2; o >= 1; o >>= 1) {
        const double os = __shfl_xor(best_score, o, 64);
        uint32_t ot = __shfl_xor(best_tag, o, 64);
        const int oj2 = __shfl_xor(best_j, o, 64);
        if (oj2 < 0) continue;
        bool take = best_j < 0 || os < best_score;
        if (!take && os == best_score) {            // tie across the group: compare tags
            if (ot == kTagUnread) ot = D.tag[oj2];
            if (best_tag == kTagUnread) best_tag = D.tag[best_j];
            take = ot < best_tag;
        }
        if (take) {
            best_score = os;
            best_tag = ot;
            best_j = oj2;
        }
    }
    tgi_out = tgi;
    return best_j;
}

// Proposal phase fused with the first matching round: proposals and their
// priority keys (Philox of the MATCH stream), posted with 64-bit atomicMin at
// both sites for round 1.  A workgroup owns 256 sites, four runs of 64
// consecutive ones (one per wave) taken from the four quarters of the index
// range, which evens out the number of sites per workgroup that can propose
// where they cluster in space (each pass of the scan below over 256 / TPP
// listed sites is a chain of dependent loads; with particles stored in
// blocks of one type, contiguous workgroups needed up to four passes in
// series while others had none).  One thread per site clears the site's
// sweep state and tests whether it can propose (a type of the reaction,
// free valence); the sites that can are listed in LDS, and then TPP threads
// per listed site scan its neighbour list.  Full or unreactive sites, most
// of a bonded system, so cost one thread each.
template <int TPP>
__global__ __launch_bounds__(256) void k_propose(const Params P, const Dev D, int slot, int xcur, int sp) {
    constexpr uint32_t kSites = 256, kPerPass = 256 / TPP;
    __shared__ uint32_t list[kSites];
    __shared__ uint32_t count;
    const unsigned long long s = D.stepv[sp];
    const int a = sweep_reaction(P, s, slot);
    const uint32_t tid = threadIdx.x;
    // run (wave * grid + workgroup) of 64 sites: a bijection of the 4 * grid
    // runs, which cover [0, n) since grid = ceil(n / 256)
    const uint32_t i0 = (((tid >> 6) * gridDim.x + xcd_block()) << 6) + (tid & 63u);
    if (blockIdx.x == 0 && tid == 0) {
        D.live_count[0] = 0u;
        if (slot == 0) {                      // a new sweep: its event lists start empty
            D.evc[0] = 0u;
            D.evc[1] = 0u;
            D.evc[2] = (uint32_t)s;
            D.evc[3] = (uint32_t)(s >> 32);
        }
    }
    if (tid == 0) count = 0u;
    __syncthreads();
    if (i0 < P.n) {
        D.best[2][i0] = kNoKey;
        D.claimed[i0] = 0;
        D.estate[i0] = kEdgeNone;
        D.prop[i0] = -1;
        const uint32_t ti = type_of(D.x[xcur][i0]);
        const uint32_t occ = D.occ[i0];
        if ((ti == P.ra[a] || ti == P.rb[a]) && occ < P.cap[ti]) list[atomicAdd(&count, 1u)] = i0;
    }
    __syncthreads();
    const uint32_t nlist = count;
    const uint32_t lane = tid % TPP;
    for (uint32_t c0 = 0; c0 < nlist; c0 += kPerPass) {
        const uint32_t p = c0 + tid / TPP;
        if (p >= nlist) break;                 // whole TPP groups leave together
        const uint32_t i = list[p];
        uint32_t tgi = 0;
        const int best_j = propose_site<TPP>(P, D, a, D.x[xcur], i, lane, tgi);
        if (lane != 0 || best_j < 0) continue;
        const unsigned long long key = match_key(P, a, s, tgi);
        D.prop[i] = best_j;
        D.key[i] = key;
        D.estate[i] = kEdgeLive;
        atomicMin(&D.best[1][i], key);
        atomicMin(&D.best[1][best_j], key);
    }
}

// What the acceptance of pair (i, j) reads: positions, tags, every slot word
// and the occupancy of both sites, loaded together.
struct PairData {
    float4 pi, pj;
    uint32_t tgi, tgj, occ_i, occ_j;
    uint32_t wi[kMaxValence], wj[kMaxValence];
};

__device__ __forceinline__ PairData load_pair(const Params& P, const Dev& D, const float4* __restrict__ X,
                                              uint32_t i, uint32_t j) {
    const size_t n = P.n;
    PairData d;
    d.pi = X[i];
    d.pj = X[j];
    d.tgi = D.tag[i];
    d.tgj = D.tag[j];
#pragma unroll
    for (int k = 0; k < kMaxValence; ++k) {
        d.wi[k] = (uint32_t)k < P.cap_max ? D.dyn[(size_t)k * n + i] : 0u;
        d.wj[k] = (uint32_t)k < P.cap_max ? D.dyn[(size_t)k * n + j] : 0u;
    }
    d.occ_i = D.occ[i];
    d.occ_j = D.occ[j];
    return d;
}

// Acceptance of a claimed pair (Eq. pon) from its loaded data: returns true
// when the bond forms, in which case both sites get the bond in their first
// free slot.
template <bool EXT>
__device__ __forceinline__ bool accept_loaded(const Params& P, const Dev& D, int a, unsigned long long s,
                                              const PairData& d, uint32_t i, uint32_t j) {
    const size_t n = P.n;
    const float4 pi = d.pi, pj = d.pj;
    const uint32_t tgi = d.tgi, tgj = d.tgj, occ_i = d.occ_i, occ_j = d.occ_j;
    const uint32_t* wi = d.wi;
    const uint32_t* wj = d.wj;
    const double kT = sweep_kT(P, D, s);
    const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
    const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
    const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
    const double r = norm3(dx, dy, dz);
    double U, pon = P.pon[a];
    if (EXT) {
        U = bond_energy(P, P.rbt[a], r);
        if (P.rmod[a] == 1u && P.kt_kinetic) pon = melt_mix(P.pon_i[a], P.pon_m[a], P.mlam[a], P.mtm[a], kT);
    } else {                                      // harmonic, the same arithmetic as bond_energy
        const double d = r - P.r0[a];
        U = P.hk[a] * (d * d);
    }
    double prob;
    if (kT > 0.0) {
        prob = pon * exp_det(-U / kT);
        prob = prob < 1.0 ? prob : 1.0;
    } else {
        prob = U <= 0.0 ? pon : 0.0;
    }
    const uint32_t lo = tgi < tgj ? tgi : tgj, hi = tgi < tgj ? tgj : tgi;
    const Word4 w = philox((uint32_t)s, (uint32_t)(s >> 32), lo, hi, P.seed, stream_k1(kOn, a, 0));
    if (!(u53(w.w0, w.w1) < prob)) return false;
    const uint32_t ti = type_of(pi), tj = type_of(pj);
    const uint32_t tagbits = ((uint32_t)a << 24) | kNewBit;
    int fi = -1, fj = -1;
#pragma unroll
    for (int k = kMaxValence - 1; k >= 0; --k) {
        if ((uint32_t)k < P.cap[ti] && wi[k] == kEmpty) fi = k;
        if ((uint32_t)k < P.cap[tj] && wj[k] == kEmpty) fj = k;
    }
    if (fi >= 0) D.dyn[(size_t)fi * n + i] = j | tagbits;
    if (fj >= 0) D.dyn[(size_t)fj * n + j] = i | tagbits;
    D.occ[i] = (uint8_t)(occ_i + 1);
    D.occ[j] = (uint8_t)(occ_j + 1);
    ev_push(P, D, 0, true, lo, hi, a);
    return true;
}

template <bool EXT>
__device__ __forceinline__ bool accept_pair(const Params& P, const Dev& D, int a, unsigned long long s,
                                            const float4* __restrict__ X, uint32_t i, uint32_t j) {
    return accept_loaded<EXT>(P, D, a, s, load_pair(P, D, X, i, j), i, j);
}

// Claim round q: a live proposal whose key is the minimum at both of its
// sites is part of the greedy matching; it is claimed and tried at once.
// The state, proposal, key and minimum at i are loaded together; where the
// key is the minimum at i, the minimum at the partner is loaded together
// with everything the acceptance reads (safe to read early: when the pair is
// claimed, no other claim touches either site, since claimed pairs share no
// site), so that a claim waits for two memory round trips.
template <bool EXT>
__global__ __launch_bounds__(256) void k_claim(const Params P, const Dev D, int slot, int q,
                                               int xcur, int sp) {
    const unsigned long long s = D.stepv[sp];
    const int a = sweep_reaction(P, s, slot);
    const uint32_t i = xcd_block() * blockDim.x + threadIdx.x;
    const unsigned long long* __restrict__ B = D.best[q % 3];
    uint32_t matched = 0, formed = 0;
    if (i < P.n) {
        const uint8_t es = D.estate[i];
        const int32_t pj = D.prop[i];
        const unsigned long long key = D.key[i];
        const unsigned long long bi = B[i];
        if (es == kEdgeLive && bi == key) {
            const uint32_t j = (uint32_t)pj;
            const unsigned long long bj = B[j];
            const PairData d = load_pair(P, D, D.x[xcur], i, j);
            if (bj == key) {
                matched = 1;
                D.estate[i] = kEdgeMatched;
                D.claimed[i] = 1;
                D.claimed[j] = 1;
                formed = accept_loaded<EXT>(P, D, a, s, d, i, j) ? 1u : 0u;
            }
        }
    }
    count_add(D, a, kCtrAttempt, matched);
    count_add(D, a, kCtrForm, formed);
}

// Kill round q: drop proposals that touch a claimed site; post the keys of
// the rest for claim round q, or, with `compact` (the last kill, before the
// finishing pass), append them with their partner and key to the live list
// instead (wave ballot + mbcnt prefix, one atomic per wave).
__global__ __launch_bounds__(256) void k_kill(const Params P, const Dev D, int q, int compact) {
    const uint32_t i = xcd_block() * blockDim.x + threadIdx.x;
    bool live = false;
    uint32_t j = 0;
    unsigned long long key = 0;
    // clear the buffer of the next kill's keys; the last kill has none (the
    // buffer it would clear is cleared again before any later use)
    if (i < P.n && !compact) D.best[(q + 1) % 3][i] = kNoKey;
    if (i < P.n && D.estate[i] == kEdgeLive) {
        j = (uint32_t)D.prop[i];
        key = D.key[i];
        if (D.claimed[i] || D.claimed[j]) {
            D.estate[i] = kEdgeDead;
        } else {
            live = true;
            if (!compact) {
                atomicMin(&D.best[q % 3][i], key);
                atomicMin(&D.best[q % 3][j], key);
            }
        }
    }
    if (compact) {
        const unsigned long long mask = __ballot(live);
        if (mask) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            const int leader = __ffsll((long long)mask) - 1;
            uint32_t base = 0;
            if (__lane_id() == leader) base = atomicAdd(D.live_count, (uint32_t)__popcll(mask));
            base = __shfl(base, leader, 64);
            if (live) D.live[base + rank] = make_uint4(i, j, (uint32_t)key, (uint32_t)(key >> 32));
        }
    }
}

// Remaining matching rounds inside one workgroup over the compacted live list.
// Every round claims at least the globally smallest live key, so the loop ends
// after at most `count` rounds.  Phases are separated by an agent-scope fence
// and a barrier so that plain loads see the atomics and stores of the phase
// before.
constexpr uint32_t kFinishLds = 256;    // live proposals matched inside LDS by k_finish

// k_finish for at most kFinishLds live proposals: the rounds run on copies in
// LDS.  An edge is claimed when no live edge sharing one of its sites has a
// smaller key; then live edges touching a claimed site die.  Claimed edges
// are vertex-disjoint and acceptance depends only on the pair, so they are
// all tried after the last round.  The list holds exactly the proposals that
// the last kill found live with both sites unclaimed, and nothing claims a
// site between that kill and this pass.
// The pair data each entry's acceptance reads is loaded before the rounds,
// overlapping them (no other entry writes the sites of a claimed pair).
template <bool EXT>
__device__ __forceinline__ void finish_in_lds(const Params& P, const Dev& D, int a, unsigned long long s,
                                              int xcur, uint32_t count) {
    __shared__ uint32_t ei[kFinishLds], ej[kFinishLds];
    __shared__ unsigned long long ek[kFinishLds];
    __shared__ uint8_t est[kFinishLds];
    __shared__ int live_left;
    const uint32_t t = threadIdx.x;
    PairData d;
    if (t < count) {
        const uint4 e = D.live[t];
        ei[t] = e.x;
        ej[t] = e.y;
        ek[t] = ((unsigned long long)e.w << 32) | e.z;
        est[t] = kEdgeLive;
        d = load_pair(P, D, D.x[xcur], e.x, e.y);
    }
    auto touches = [&](uint32_t e, uint32_t f) {
        return ei[f] == ei[e] || ei[f] == ej[e] || ej[f] == ei[e] || ej[f] == ej[e];
    };
    for (uint32_t round = 0; round <= count; ++round) {
        __syncthreads();                 // everyone has read live_left of the last round
        if (t == 0) live_left = 0;
        __syncthreads();
        bool win = false;
        if (t < count && est[t] == kEdgeLive) {
            win = true;
            for (uint32_t f = 0; f < count; ++f)
                if (f != t && est[f] == kEdgeLive && ek[f] < ek[t] && touches(t, f)) { win = false; break; }
        }
        __syncthreads();
        if (win) est[t] = kEdgeMatched;
        __syncthreads();
        if (t < count && est[t] == kEdgeLive) {
            for (uint32_t f = 0; f < count; ++f)
                if (est[f] == kEdgeMatched && touches(t, f)) { est[t] = kEdgeDead; break; }
            if (est[t] == kEdgeLive) live_left = 1;
        }
        __syncthreads();
        if (!live_left) break;
    }
    uint32_t att = 0, form = 0;
    if (t < count) {
        const uint32_t i = ei[t], j = ej[t];
        if (est[t] == kEdgeMatched) {
            D.estate[i] = kEdgeMatched;
            D.claimed[i] = 1;
            D.claimed[j] = 1;
            att = 1;
            form = accept_loaded<EXT>(P, D, a, s, d, i, j) ? 1u : 0u;
        } else {
            D.estate[i] = kEdgeDead;
        }
    }
    if (t < kFinishLds) {
        count_add(D, a, kCtrAttempt, att);
        count_add(D, a, kCtrForm, form);
    }
}

template <bool EXT>
__global__ __launch_bounds__(1024) void k_finish(const Params P, const Dev D, int slot, int buf,
                                                 int xcur, int sp, uint32_t lds_limit) {
    const unsigned long long s = D.stepv[sp];
    const int a = sweep_reaction(P, s, slot);
    unsigned long long* B = D.best[buf];
    const uint32_t count = D.live_count[0];
    if (count <= lds_limit && count <= kFinishLds) {
        finish_in_lds<EXT>(P, D, a, s, xcur, count);
        return;
    }
    __shared__ int any;
    __shared__ uint32_t n_att, n_form;
    if (threadIdx.x == 0) { n_att = 0; n_form = 0; }
    for (uint32_t round = 0; round <= count; ++round) {
        __syncthreads();
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < count; e += blockDim.x) {
            const uint32_t i = D.live[e].x;
            if (D.estate[i] != kEdgeLive) continue;
            const uint32_t j = (uint32_t)D.prop[i];
            if (D.claimed[i] || D.claimed[j]) {
                D.estate[i] = kEdgeDead;
                continue;
            }
            atomicMin(&B[i], D.key[i]);
            atomicMin(&B[j], D.key[i]);
            any = 1;
        }
        __threadfence();
        __syncthreads();
        if (!any) break;
        for (uint32_t e = threadIdx.x; e < count; e += blockDim.x) {
            const uint32_t i = D.live[e].x;
            if (D.estate[i] != kEdgeLive) continue;
            const uint32_t j = (uint32_t)D.prop[i];
            const unsigned long long key = D.key[i];
            if (B[i] == key && B[j] == key) {
                D.estate[i] = kEdgeMatched;
                D.claimed[i] = 1;
                D.claimed[j] = 1;
                atomicAdd(&n_att, 1u);
                if (accept_pair<EXT>(P, D, a, s, D.x[xcur], i, j)) atomicAdd(&n_form, 1u);
            }
        }
        __threadfence();
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < count; e += blockDim.x) {
            const uint32_t i = D.live[e].x;
            B[i] = kNoKey;
            B[(uint32_t)D.prop[i]] = kNoKey;
        }
        __threadfence();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (n_att) atomicAdd(ctr_slot(D, a, kCtrAttempt, 0), (unsigned long long)n_att);
        if (n_form) atomicAdd(ctr_slot(D, a, kCtrForm, 0), (unsigned long long)n_form);
    }
}

// Breaking at site i for reaction a (sweep at step s): bonds of reaction a
// present at the start of the sweep break with P0_off; bonds formed in this
// sweep only lose their "new" mark.  Each site edits its own slots; both ends
// draw the same number.  All slot words are loaded at once, then the
// partners' tags.  Returns the number of bonds broken with i as the lower tag.
template <bool EXT>
__device__ __forceinline__ uint32_t break_site(const Params& P, const Dev& D, int a, unsigned long long s,
                                               uint32_t i, const float4* __restrict__ X) {
    const size_t n = P.n;
    uint32_t broke = 0;
    uint32_t w[kMaxValence];
    bool mine[kMaxValence];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kMaxValence; ++k) {
        w[k] = (uint32_t)k < P.cap_max ? D.dyn[(size_t)k * n + i] : kEmpty;
        mine[k] = w[k] != kEmpty && ((w[k] >> 24) & 0x7Fu) == (uint32_t)a;
        any |= mine[k];
    }
    if (!any) return 0u;
    const uint32_t tgi = D.tag[i];
    uint32_t tgj[kMaxValence];
#pragma unroll
    for (int k = 0; k < kMaxValence; ++k)     // unconditional (clamped) loads, issued together
        tgj[k] = D.tag[mine[k] ? (w[k] & kIdxMask) : i];
    uint32_t occ = D.occ[i];
    const uint32_t occ0 = occ;
    // rate modifiers: the melted P0_off at the kinetic temperature, or the
    // slip factor from each bond's length (both ends compute the same r)
    const uint32_t mod = EXT ? P.rmod[a] : 0u;
    double poff = P.poff[a], kT = 0.0;
    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
    if (mod != 0u) {
        kT = sweep_kT(P, D, s);
        if (mod == 1u && P.kt_kinetic) poff = melt_mix(P.poff_i[a], P.poff_m[a], P.mlam[a], P.mtm[a], kT);
        if (mod == 2u) pi = X[i];
    }
#pragma unroll
    for (int k = 0; k < kMaxValence; ++k) {
        if (!mine[k]) continue;
        uint32_t* sl = &D.dyn[(size_t)k * n + i];
        if (w[k] & kNewBit) { *sl = w[k] & ~kNewBit; continue; }
        const uint32_t lo = tgi < tgj[k] ? tgi : tgj[k], hi = tgi < tgj[k] ? tgj[k] : tgi;
        const Word4 r = philox((uint32_t)s, (uint32_t)(s >> 32), lo, hi, P.seed, stream_k1(kOff, a, 0));
        double q = poff;
        if (mod == 2u) {
            const float4 pj = X[w[k] & kIdxMask];
            const double dx = mi_delta(pi.x, pj.x, P.L, P.invL);
            const double dy = mi_delta(pi.y, pj.y, P.L, P.invL);
            const double dz = mi_delta(pi.z, pj.z, P.L, P.invL);
            q = slip_prob(poff, P.slip[a], bond_energy(P, P.rbt[a], norm3(dx, dy, dz)), kT);
        }
        const bool gone = u53(r.w0, r.w1) < q;
        if (gone) {
            *sl = kEmpty;
            --occ;
            if (tgi < tgj[k]) ++broke;
        }
        ev_push(P, D, 1, gone && tgi < tgj[k], lo, hi, a);   // listed once, by the lower tag
    }
    if (occ != occ0) D.occ[i] = (uint8_t)occ;
    return broke;
}

// Breaking phase (Sec. 2.3, Fig. sweep d), one thread per site (break_site).
// Also resets best[1] for the next reaction's proposal round.
template <bool EXT>
__global__ __launch_bounds__(256) void k_break(const Params P, const Dev D, int slot, int xcur, int sp,
                                               int last) {
    const unsigned long long s = D.stepv[sp];
    const int a = sweep_reaction(P, s, slot);
    const uint32_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (last && i == 0) D.ke_fix[ke_slot(P, s) ^ 1u] = 0ull;   // the next sweep's slot
    uint32_t broke = 0;
    if (i < P.n) {
        D.best[1][i] = kNoKey;
        broke = break_site<EXT>(P, D, a, s, i, D.x[xcur]);
    }
    count_add(D, a, kCtrBreak, broke);
}

// ------------------------------------------------------------ I/O kernels
// Gather index-ordered float4 (positions, u, or f4 + h F/m) into tag order.
// mode 0: positions, 1: full-step velocities (u + h F/m, F in f4), 2: forces (f4)
__global__ void k_gather(const Params P, const Dev D, float4* __restrict__ out, int xin, int mode) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    const uint32_t i = D.rtag[t];
    if (mode == 0) {
        out[t] = D.x[xin][i];
    } else if (mode == 1) {
        const float hm = P.h * P.inv_mass[type_of(D.x[xin][i])];
        const float4 u = D.u[i], f = D.f4[i];
        out[t] = make_float4(u.x + hm * f.x, u.y + hm * f.y, u.z + hm * f.z, 0.0f);
    } else {
        out[t] = D.f4[i];
    }
}
// The same read-outs as k_gather, as x, y, z triplets in tag order into
// caller memory (out3 holds 3 n floats).
__global__ void k_gather3(const Params P, const Dev D, float* __restrict__ out3, int xin, int mode) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    const uint32_t i = D.rtag[t];
    float4 v;
    if (mode == 0) {
        v = D.x[xin][i];
    } else if (mode == 1) {
        const float hm = P.h * P.inv_mass[type_of(D.x[xin][i])];
        const float4 u = D.u[i], f = D.f4[i];
        v = make_float4(u.x + hm * f.x, u.y + hm * f.y, u.z + hm * f.z, 0.0f);
    } else {
        v = D.f4[i];
    }
    out3[3 * (size_t)t] = v.x;
    out3[3 * (size_t)t + 1] = v.y;
    out3[3 * (size_t)t + 2] = v.z;
}
__global__ void k_gather_img(const Params P, const Dev D, int32_t* __restrict__ out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    const uint32_t i = D.rtag[t];
    out[3 * t + 0] = D.img[i];
    out[3 * t + 1] = D.img[P.n + i];
    out[3 * t + 2] = D.img[2 * P.n + i];
}

// Energies and bond counts: red[0] = PE, red[1] = KE (2^-32 fixed point),
// red[2 + a] = bonds of reaction a.
__global__ __launch_bounds__(256) void k_observe(const Params P, const Dev D, int xin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ uint32_t nb[kMaxRx];
    if (threadIdx.x < kMaxRx) nb[threadIdx.x] = 0u;
    __syncthreads();
    unsigned long long pe = 0, ke = 0;
    if (i < P.n) {
        const uint32_t ti = type_of(D.x[xin][i]);
        const float4 f = D.f4[i];
        const float4 u = D.u[i];
        const float hm = P.h * P.inv_mass[ti];
        const double vx = u.x + hm * f.x, vy = u.y + hm * f.y, vz = u.z + hm * f.z;
        pe = (unsigned long long)rint((double)f.w * 4294967296.0);
        ke = (unsigned long long)rint(0.5 * (double)P.mass[ti] * ((vx * vx + vy * vy) + vz * vz) * 4294967296.0);
        const uint32_t tgi = D.tag[i];
        for (uint32_t k = 0; k < P.cap[ti]; ++k) {
            const uint32_t w = D.dyn[(size_t)k * P.n + i];
            if (w == kEmpty) continue;
            if (D.tag[w & kIdxMask] > tgi) atomicAdd(&nb[(w >> 24) & 0x7Fu], 1u);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        pe += __shfl_xor(pe, off, 64);
        ke += __shfl_xor(ke, off, 64);
    }
    if (__lane_id() == 0) {
        atomicAdd(&D.red[0], pe);
        atomicAdd(&D.red[1], ke);
    }
    __syncthreads();
    if (threadIdx.x < P.nrx && nb[threadIdx.x]) atomicAdd(&D.red[2 + threadIdx.x], (unsigned long long)nb[threadIdx.x]);
}

// Connected components over static + dynamic bonds (union by minimum index).
__device__ __forceinline__ uint32_t cc_root(const uint32_t* parent, uint32_t v) {
    uint32_t p = parent[v];
    while (p != v) { v = p; p = parent[v]; }
    return v;
}
__global__ void k_cc_init(const Params P, const Dev D) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) D.parent[i] = i;
}
__device__ __forceinline__ void cc_hook_edge(const Dev& D, uint32_t i, uint32_t j, uint32_t* changed) {
    if (j < i) return;                     // each edge once, from its lower index
    const uint32_t ri = cc_root(D.parent, i), rj = cc_root(D.parent, j);
    if (ri == rj) return;
    atomicMin(&D.parent[ri < rj ? rj : ri], ri < rj ? ri : rj);
    *changed = 1u;
}
__global__ void k_cc_hook(const Params P, const Dev D, uint32_t* changed, int xin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    for (uint32_t k = 0; k < P.stat_max; ++k) {
        const uint32_t w = D.stat[(size_t)k * P.n + i];
        if (w == kEmpty) break;
        cc_hook_edge(D, i, w & kIdxMask, changed);
    }
    const uint32_t cap = P.cap[type_of(D.x[xin][i])];
    for (uint32_t k = 0; k < cap; ++k) {
        const uint32_t w = D.dyn[(size_t)k * P.n + i];
        if (w != kEmpty) cc_hook_edge(D, i, w & kIdxMask, changed);
    }
}
__global__ void k_cc_compress(const Params P, const Dev D) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) D.parent[i] = cc_root(D.parent, i);
}
__global__ void k_cc_size(const Params P, const Dev D) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) atomicAdd(&D.scan[D.parent[i]], 1u);
}
__global__ void k_cc_max(const Params P, const Dev D) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n && D.scan[i]) atomicMax((unsigned long long*)&D.red[2 + kMaxRx], (unsigned long long)D.scan[i]);
}

// ------------------------------------------------------------ network analyses
// Clusters of size k (k < len) in hist[k - 1], larger ones in hist[len - 1];
// D.scan holds each root's cluster size (k_cc_size).
__global__ void k_cc_hist(const Params P, const Dev D, unsigned long long* hist, uint32_t len,
                          unsigned long long* n_clusters) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const uint32_t k = D.scan[i];
    if (k == 0u) return;
    atomicAdd(&hist[(k < len ? k : len) - 1u], 1ull);
    atomicAdd(n_clusters, 1ull);
}

// Reference bond table for the bond correlation, by tag: slot c of tag t
// holds the c-th bond of t to a higher tag as partner tag | reaction << 24
// (tags and indices are below 2^24).
__global__ void k_bond_ref(const Params P, const Dev D, uint32_t* __restrict__ ref, int xin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const size_t n = P.n;
    const uint32_t t = D.tag[i];
    const uint32_t cap = P.cap[type_of(D.x[xin][i])];
    uint32_t c = 0;
    for (uint32_t k = 0; k < cap; ++k) {
        const uint32_t w = D.dyn[(size_t)k * n + i];
        if (w == kEmpty) continue;
        const uint32_t tj = D.tag[w & kIdxMask];
        if (tj > t) ref[(size_t)c++ * n + t] = tj | (((w >> 24) & 0x7Fu) << 24);
    }
    for (; c < P.cap_max; ++c) ref[(size_t)c * n + t] = kEmpty;
}

// Reference bonds (out[0]) and those present now between the same two
// sites with the same reaction (out[1]); one thread per tag.
__global__ __launch_bounds__(256) void k_bond_corr(const Params P, const Dev D, const uint32_t* __restrict__ ref,
                                                   unsigned long long* out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nref = 0, kept = 0;
    if (t < P.n) {
        const size_t n = P.n;
        const uint32_t i = D.rtag[t];
        for (uint32_t c = 0; c < P.cap_max; ++c) {
            const uint32_t w = ref[(size_t)c * n + t];
            if (w == kEmpty) continue;
            ++nref;
            const uint32_t j = D.rtag[w & kIdxMask], a = (w >> 24) & 0x7Fu;
            for (uint32_t k = 0; k < P.cap_max; ++k) {
                const uint32_t d = D.dyn[(size_t)k * n + i];
                if (d != kEmpty && (d & kIdxMask) == j && ((d >> 24) & 0x7Fu) == a) {
                    ++kept;
                    break;
                }
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        nref += __shfl_xor(nref, off, 64);
        kept += __shfl_xor(kept, off, 64);
    }
    if (__lane_id() == 0 && nref) {
        atomicAdd(&out[0], nref);
        atomicAdd(&out[1], kept);
    }
}

// Dynamic bonds per pair of molecules, counted in an open-addressing table
// (keys: lower molecule id << 32 | higher one; ~0 = empty; size mask + 1, a
// power of two above the number of bonds, so every probe sequence ends);
// bonds inside one molecule go to intra[0].
__global__ __launch_bounds__(256) void k_mol_pairs(const Params P, const Dev D, int xin,
                                                   unsigned long long* __restrict__ keys,
                                                   uint32_t* __restrict__ counts, uint32_t mask,
                                                   unsigned long long* intra) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const size_t n = P.n;
    const uint32_t tgi = D.tag[i], mi = D.mol[i];
    const uint32_t cap = P.cap[type_of(D.x[xin][i])];
    for (uint32_t k = 0; k < cap; ++k) {
        const uint32_t w = D.dyn[(size_t)k * n + i];
        if (w == kEmpty) continue;
        const uint32_t j = w & kIdxMask;
        if (D.tag[j] <= tgi) continue;                       // each bond once
        const uint32_t mj = D.mol[j];
        if (mj == mi) {
            atomicAdd(intra, 1ull);
            continue;
        }
        const unsigned long long key = ((unsigned long long)(mi < mj ? mi : mj) << 32) | (mi < mj ? mj : mi);
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
        for (;;) {
            const unsigned long long prev = atomicCAS(&keys[h], ~0ull, key);
            if (prev == ~0ull || prev == key) {
                atomicAdd(&counts[h], 1u);
                break;
            }
            h = (h + 1u) & mask;
        }
    }
}

// Histogram of the table's counts: pairs joined by m bonds in hist[m - 1]
// (m < len), by len or more in hist[len - 1]; pairs in n_pairs.
__global__ void k_mol_hist(const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ counts,
                           uint32_t size, unsigned long long* hist, uint32_t len, unsigned long long* n_pairs) {
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= size || keys[h] == ~0ull) return;
    const uint32_t m = counts[h];
    atomicAdd(&hist[(m < len ? m : len) - 1u], 1ull);
    atomicAdd(n_pairs, 1ull);
}

// Bond read-out, in tag order.  Pass 1: per tag, the number of its dynamic
// bonds to a higher tag, exclusive-scanned inside each block (wave shuffles),
// block totals to `bsum`.  Pass 2 scans `bsum`; pass 3 writes the rows.
__device__ __forceinline__ int rows_of(const Params& P, const Dev& D, int xin, uint32_t t, uint32_t* ptag,
                                       uint32_t* pbt) {
    const uint32_t i = D.rtag[t];
    const uint32_t ti = type_of(D.x[xin][i]);
    int c = 0;
    for (uint32_t k = 0; k < P.cap[ti]; ++k) {
        const uint32_t w = D.dyn[(size_t)k * P.n + i];
        if (w == kEmpty) continue;
        const uint32_t tj = D.tag[w & kIdxMask];
        if (tj <= t) continue;
        if (ptag) {
            const uint32_t bt = P.rbt[(w >> 24) & 0x7Fu];
            int p = c;   // insertion sort by (partner tag, bond type)
            while (p > 0 && (ptag[p - 1] > tj || (ptag[p - 1] == tj && pbt[p - 1] > bt))) {
                ptag[p] = ptag[p - 1];
                pbt[p] = pbt[p - 1];
                --p;
            }
            ptag[p] = tj;
            pbt[p] = bt;
        }
        ++c;
    }
    return c;
}

__global__ __launch_bounds__(256) void k_rows_count(const Params P, const Dev D, int xin, uint32_t* bsum) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = t < P.n ? (uint32_t)rows_of(P, D, xin, t, nullptr, nullptr) : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(c, &tot);
    if (t < P.n) D.scan[t] = ex;
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_bsum(uint32_t* bsum, uint32_t nb) {
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += blockDim.x) {
        const uint32_t k = base + threadIdx.x;
        const uint32_t v = k < nb ? bsum[k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, &tot);
        const uint32_t c0 = carry;
        if (k < nb) bsum[k] = c0 + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(256) void k_rows_emit(const Params P, const Dev D, int xin, const uint32_t* bsum,
                                                   uint32_t* pairs, uint32_t* btypes) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    uint32_t ptag[kMaxValence], pbt[kMaxValence];
    const int c = rows_of(P, D, xin, t, ptag, pbt);
    const uint32_t at = bsum[blockIdx.x] + D.scan[t];
    for (int k = 0; k < c; ++k) {
        pairs[2 * (at + k)] = t;
        pairs[2 * (at + k) + 1] = ptag[k];
        btypes[at + k] = pbt[k];
    }
}

}  // namespace dyb
