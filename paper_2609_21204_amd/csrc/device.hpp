// Device-side building blocks of the dynamic-bonding MD step (gfx950).
//
// Counter-based random numbers (Philox4x32-10, Salmon et al. SC'11), the
// FP64 geometry that every bond decision is taken with, and the parameter
// and state blocks passed to every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dyb {

constexpr int kMaxTypes = 8;
constexpr int kMaxRx = 8;
constexpr int kMaxBondTypes = 8;
constexpr int kMaxValence = 8;
constexpr int kMaxStatic = 8;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;       // empty bond slot
constexpr uint32_t kIdxMask = 0x00FFFFFFu;     // partner index bits of a slot word
constexpr uint32_t kNewBit = 0x80000000u;      // dynamic bond formed in the running sweep
constexpr uint64_t kNoKey = ~0ull;
constexpr float kFixScale = 4294967296.0f;     // 2^32: fixed-point force / energy scale
constexpr double kFixInv = 1.0 / 4294967296.0;

// Random stream kinds: one stream per purpose, reaction and replica.
enum : uint32_t { kThermo = 1, kOrder = 2, kMatch = 3, kOn = 4, kOff = 5, kInit = 6 };

// Edge states of the matching phase.
enum : uint8_t { kEdgeNone = 0, kEdgeLive = 1, kEdgeMatched = 2, kEdgeDead = 3 };

// Device error flags (sticky until the host clears them).
enum : uint32_t { kErrOverflow = 1u, kErrFene = 2u, kErrForce = 4u, kErrNlist = 8u };   // kErrFene: a bond outside its range

// ---------------------------------------------------------------- Philox
struct Word4 { uint32_t w0, w1, w2, w3; };

// Philox4x32 with 10 rounds.  A round multiplies counter words 0 and 2 by
// the two round constants, swaps the halves into the other two words xor-ed
// with the key, and bumps the key by the Weyl increments.
__host__ __device__ inline Word4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Word4{c0, c1, c2, c3};
}

__host__ __device__ inline uint32_t stream_k1(uint32_t kind, uint32_t rx, uint32_t replica) {
    return (kind << 24) | (rx << 16) | (replica & 0xFFFFu);
}

// 53-bit uniform double in [0, 1).
__host__ __device__ inline double u53(uint32_t w0, uint32_t w1) {
    const uint64_t bits = ((uint64_t)w0 << 21) | (uint64_t)(w1 >> 11);
    return (double)bits * 0x1.0p-53;
}

// Random processing order of the reactions of the sweep at step s: Fisher-
// Yates from the last slot down, slot k swapped with floor(w (k+1) / 2^32),
// words taken in order from Philox blocks (s, 0, block) of the ORDER stream.
// Returns the reaction processed in slot `slot`.
__host__ __device__ inline int reaction_at(uint32_t seed, uint64_t s, int nrx, int slot) {
    int order[kMaxRx];
    for (int k = 0; k < nrx; ++k) order[k] = k;
    if (nrx > 1) {
        const uint32_t k1 = stream_k1(kOrder, 0, 0);
        Word4 blk{};
        int used = 4;
        uint32_t block = 0;
        for (int k = nrx - 1; k >= 1; --k) {
            if (used == 4) {
                blk = philox((uint32_t)s, (uint32_t)(s >> 32), 0u, block++, seed, k1);
                used = 0;
            }
            const uint32_t w = used == 0 ? blk.w0 : used == 1 ? blk.w1 : used == 2 ? blk.w2 : blk.w3;
            ++used;
            const int j = (int)(((uint64_t)w * (uint64_t)(k + 1)) >> 32);
            const int t = order[k];
            order[k] = order[j];
            order[j] = t;
        }
    }
    return order[slot];
}

// ---------------------------------------------------------------- decision math
// exp, log1p and tanh for what decides bonds: the acceptance factor of
// Eq. pon, the slip factor of Eq. slip, the melting switch of Eq. gT and the
// FENE and tether bond energies.  Only IEEE-rounded +, -, *, / and exact
// power-of-two scaling, in a fixed order with contraction off, so every
// device and the host produce the same bits for the same input (and so does
// any other implementation of these same steps); a few ulp from the exact
// functions.
//   exp:   Cody-Waite reduction (Cody & Waite, 1980): n = rint(x / ln2), ln2
//          split into a head of 29 bits (n head is exact) and a tail,
//          r = (x - n head) - n tail; Taylor series of e^r to degree 13 by
//          Horner; times 2^n.
//   log1p: 1 + z = m 2^e, m in [sqrt(1/2), sqrt(2)); s = (m - 1)/(m + 1), or
//          z / (2 + z) when e = 0 (small z keep their bits); log m by the
//          atanh series 2 (s + s^3/3 + ... + s^23/23) in Horner form in s^2;
//          plus e head + e tail.
//   tanh:  1 - 2 / (exp(2|x|) + 1) with the sign of x, 1 beyond |x| = 22.
constexpr double kLn2Hi = 0x1.62e42fe000000p-1;
constexpr double kLn2Lo = 0x1.f473de6af278fp-30;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;

__host__ __device__ inline double exp_det(double x) {
#pragma clang fp contract(off)
    if (x != x) return x;
    if (!(x > -745.5)) return 0.0;
    if (x > 709.78) return __builtin_huge_val();
    const double n = rint(x * kInvLn2);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    double p = 0x1.6124613a86d09p-33;        // 1/13!
    p = p * r + 0x1.1eed8eff8d898p-29;       // 1/12!
    p = p * r + 0x1.ae64567f544e4p-26;       // 1/11!
    p = p * r + 0x1.27e4fb7789f5cp-22;       // 1/10!
    p = p * r + 0x1.71de3a556c734p-19;       // 1/9!
    p = p * r + 0x1.a01a01a01a01ap-16;       // 1/8!
    p = p * r + 0x1.a01a01a01a01ap-13;       // 1/7!
    p = p * r + 0x1.6c16c16c16c17p-10;       // 1/6!
    p = p * r + 0x1.1111111111111p-7;        // 1/5!
    p = p * r + 0x1.5555555555555p-5;        // 1/4!
    p = p * r + 0x1.5555555555555p-3;        // 1/3!
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)n);
}

__host__ __device__ inline double log1p_det(double z) {
#pragma clang fp contract(off)
    if (z != z) return z;
    if (!(z > -1.0)) return z == -1.0 ? -__builtin_huge_val() : __builtin_nan("");
    const double y = 1.0 + z;
    int e = 0;
    double m = frexp(y, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {          // sqrt(1/2)
        m = m * 2.0;
        e -= 1;
    }
    double s;
    if (e == 0) {
        s = z / (2.0 + z);
    } else {
        const double f = m - 1.0;
        s = f / (2.0 + f);
    }
    const double s2 = s * s;
    double t = 1.0 / 23.0;
    t = t * s2 + 1.0 / 21.0;
    t = t * s2 + 1.0 / 19.0;
    t = t * s2 + 1.0 / 17.0;
    t = t * s2 + 1.0 / 15.0;
    t = t * s2 + 1.0 / 13.0;
    t = t * s2 + 1.0 / 11.0;
    t = t * s2 + 1.0 / 9.0;
    t = t * s2 + 1.0 / 7.0;
    t = t * s2 + 1.0 / 5.0;
    t = t * s2 + 1.0 / 3.0;
    const double lm = 2.0 * s + (2.0 * s) * (s2 * t);
    const double de = (double)e;
    return de * kLn2Hi + (lm + de * kLn2Lo);
}

__host__ __device__ inline double tanh_det(double x) {
#pragma clang fp contract(off)
    if (x != x) return x;
    const double a = fabs(x);
    double t = 1.0;
    if (a < 22.0) t = 1.0 - 2.0 / (exp_det(2.0 * a) + 1.0);
    return x < 0.0 ? -t : t;
}

// ---------------------------------------------------------------- geometry
// Minimum-image separation x_j - x_i in FP64 from FP32 coordinates.  The
// evaluation order is fixed and never contracted into FMAs, so that every
// bond decision sees exactly the same r on every device and on the host.
__device__ __forceinline__ double mi_delta(float xi, float xj, double L, double invL) {
#pragma clang fp contract(off)
    const double d = (double)xj - (double)xi;
    const double q = d * invL;
    if (!(fabs(q) > 0.5)) return d;       // rint(q) == 0: no image (d - 0 L == d)
    return d - rint(q) * L;
}

__device__ __forceinline__ double norm3(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    return sqrt(r2);
}

// ---------------------------------------------------------------- blocks
struct Params {
    uint32_t tile[3];      // cells per tile along x, y, z (core of one k_step workgroup)
    uint32_t ntile[3];     // tiles along x, y, z
    uint32_t n, ntypes, nrx, cap_max;
    uint32_t stat_max, nc, ncell, cellcap;
    uint32_t seed, period, kt_kinetic, any_self_avoid;
    double L, invL;
    float Lf, halfLf, cell_scale, h;   // h = dt / 2
    float c1;                          // exp(-gamma dt)
    uint32_t tpp;                      // threads per particle in k_propose (host side: launch shape)
    uint32_t tpp_step;                 // threads per particle in k_step
    uint32_t qb_step;                  // list entries per thread issued up front in k_step (0: by TPP)
    uint32_t ext;                      // tether bonds or rate modifiers present: kernels in their full variant
    float disp2;                       // (skin / 2 - 1e-4 - packing error of xref)^2: displacement that triggers a rebuild
    float xq, xqinv;                   // 2^21 / L and L / 2^21: the 21-bit grid of the packed build positions
    uint32_t nlmax;                    // neighbour-list slots per particle
    uint32_t evcap[2];                 // capacity of the formed / broken event lists of a sweep
    double kT;
    float inv_mass[kMaxTypes];
    float noise_sd[kMaxTypes];         // sqrt(1 - c1^2) sqrt(kT / m)
    float mass[kMaxTypes];
    uint32_t cap[kMaxTypes];
    float rc2_pre[kMaxTypes * kMaxTypes];  // FP32 prefilter: (2^(1/6) sigma_ij)^2 (1 + 1e-3) + 1e-4; 0 = no WCA
    float rc2_in[kMaxTypes * kMaxTypes];   // (0.98 rc)^2: below it the FP32 force has no cancellation
    float rl2[kMaxTypes * kMaxTypes];      // neighbour-list radius^2 of the type pair: (max(rc, r_max) + skin)^2 (1 + 1e-4)
    float sig2f[kMaxTypes * kMaxTypes];    // sigma_ij^2
    float eps24f[kMaxTypes * kMaxTypes];   // 24 eps_ij

    uint32_t bkind[kMaxBondTypes];     // 0 harmonic, 1 FENE, 2 tether
    double bk[kMaxBondTypes], br0[kMaxBondTypes], bR02[kMaxBondTypes], binvR02[kMaxBondTypes];
    double blmin[kMaxBondTypes], blc1[kMaxBondTypes], blc0[kMaxBondTypes], blmax[kMaxBondTypes];  // tether
    float rmax2_pre[kMaxRx], rmin2_pre[kMaxRx];  // FP32 prefilter of the reaction window
    uint32_t ra[kMaxRx], rb[kMaxRx], rbt[kMaxRx], rself[kMaxRx];
    double rmin[kMaxRx], rmax[kMaxRx], r0[kMaxRx], hk[kMaxRx], pon[kMaxRx], poff[kMaxRx];
    // rate modifiers (0 none, 1 melting, 2 slip bond).  With the set-point
    // temperature the melted probabilities are already in pon / poff; with the
    // kinetic temperature the sweep mixes pon_i / pon_m (poff_i / poff_m) by
    // the switch at that temperature.
    uint32_t rmod[kMaxRx];
    double mlam[kMaxRx], mtm[kMaxRx], pon_i[kMaxRx], pon_m[kMaxRx], poff_i[kMaxRx], poff_m[kMaxRx];
    double slip[kMaxRx];
};

// WCA parameters of one type pair, evaluated in FP64.
struct PairTab {
    double sig2;   // sigma_ij^2
    double eps24;  // 24 eps_ij
    double rc;     // 2^(1/6) sigma_ij (0: no WCA)
    double rc2_lo, rc2_hi;   // rc^2 (1 -/+ 1e-14): r < rc is decided without sqrt outside this band
    double eps;    // eps_ij
    double pad0, pad1;
};

// Per-type and per-type-pair constants of the step kernel, built on the host
// at commit and staged in LDS by every workgroup: the force loop indexes them
// with lane-varying types, which from the kernel-argument block would be one
// more dependent memory round trip per neighbour.
struct alignas(16) StepTabs {
    float rc2_pre[kMaxTypes * kMaxTypes], rc2_in[kMaxTypes * kMaxTypes];
    float sig2f[kMaxTypes * kMaxTypes], eps24f[kMaxTypes * kMaxTypes];
    float rl2[kMaxTypes * kMaxTypes];   // neighbour-list radius^2 of the type pair
    PairTab pair[kMaxTypes * kMaxTypes];
    double bk[kMaxBondTypes], br0[kMaxBondTypes], binvR02[kMaxBondTypes];
    double blmin[kMaxBondTypes], blc1[kMaxBondTypes], blc0[kMaxBondTypes], blmax[kMaxBondTypes];
    uint32_t bkind[kMaxBondTypes];
    uint32_t rbt[kMaxRx];
    float hm[kMaxTypes], noise_sd[kMaxTypes], mass[kMaxTypes];   // hm = (dt / 2) / m
    uint32_t cap[kMaxTypes];
};
static_assert(sizeof(StepTabs) % 16 == 0, "staged in 16-byte words");

struct Dev {
    const PairTab* pair;   // kMaxTypes x kMaxTypes
    const StepTabs* tabs;  // the same constants for k_step
    float4* x[2];          // positions (xyz) + type bits (w), double-buffered
    float4* u;             // velocity before the closing half kick of the last step
    int32_t* img;          // image counters, 3 x n
    uint32_t* tag;         // tag of the particle at each index
    uint32_t* rtag;        // index of each tag
    uint8_t* occ;          // dynamic-bond count per site
    uint32_t* dyn;         // cap_max x n dynamic slots: partner | rx << 24 | new bit
    uint32_t* stat;        // stat_max x n static slots: partner | bond type << 24
    uint32_t* mol;         // molecule id (static-bond component)
    uint32_t* ccount[3];   // per-cell counts of three rotating cell lists
    float4* cpos[3];       // per-cell members: position + (index | type << 24) bits, cellcap slots per cell (cell_slot)
    int32_t* prop;         // proposed partner index (-1 none)
    unsigned long long* key;        // matching priority of each proposal
    unsigned long long* best[3];    // per-site minimum key of live incident proposals (3 rotating)
    uint8_t* estate;       // proposal state
    uint8_t* claimed;      // site claimed in the running reaction
    uint4* live;           // compacted live proposals handed to the finishing pass: {i, j, key lo, key hi}
    uint32_t* live_count;  // [0] = length of `live`
    uint2* ev[2];          // bonds formed [0] and broken [1] in the last sweep: {tag_lo, tag_hi | rx << 24}
    uint32_t* evc;         // [0], [1] lengths of ev[0], ev[1]; [2], [3] step key of that sweep (lo, hi)
    unsigned long long* counters;   // nrx x 3 x kCtrSlots: attempts, forms, breaks
    unsigned long long* stepv;      // two step slots (parity of the step)
    unsigned long long* ke_fix;     // [2] sum m v^2 in 2^-32 fixed point (kinetic kT), one slot per sweep parity
    uint32_t* err;         // [0] flags, [1], [2] tags of the offending pair
    float4* f4;            // forces + per-particle energy (evaluation kernels)
    unsigned long long* red;        // reduction scratch (observables)
    uint32_t* scan;        // scan scratch (bond read-out)
    uint32_t* parent;      // union-find parents (cluster observable)
    uint32_t* nl;          // nlmax x n neighbour indices (slot-major)
    uint32_t* nl_cnt;      // neighbours per particle
    uint2* xref;           // positions at the last neighbour-list build, 21 bits per axis (xref_pack)
    uint32_t* rflag;       // neighbour-list rebuild flags of steps t, t+1, t+2 (index step mod 3);
                           // [3]: the cell list (0 or 1) the next build bins into;
                           // [4]: neighbour-list builds by db_step since commit
    uint32_t* corder;      // cells in Morton order (the renumbering's cell sequence)
    // spatial reordering (counting sort by cell): new index of every particle,
    // cell offsets, and second copies of every per-particle array
    uint32_t* newidx;
    uint32_t* cstart;      // ncell + 1
    uint32_t* cbsum;       // block sums of the cell-offset scan
    float4* x_alt;
    float4* u_alt;
    int32_t* img_alt;
    uint32_t* tag_alt;
    uint8_t* occ_alt;
    uint32_t* mol_alt;
    uint32_t* dyn_alt;
    uint32_t* stat_alt;
};

__device__ __forceinline__ uint32_t type_of(const float4& p) { return __float_as_uint(p.w); }

// Cell-slot word: particle index in the low 24 bits, type in the high 8.
__device__ __forceinline__ uint32_t slot_index(const float4& q) { return __float_as_uint(q.w) & kIdxMask; }
__device__ __forceinline__ uint32_t slot_type(const float4& q) { return __float_as_uint(q.w) >> 24; }

__device__ __forceinline__ int cell_coord(float x, const Params& P) {
    int c = (int)floorf((x + P.halfLf) * P.cell_scale);
    c = c < 0 ? 0 : c;
    return c >= (int)P.nc ? (int)P.nc - 1 : c;
}

__device__ __forceinline__ int wrapc(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// Slot k of cell c in a cell list's member array.  Slot-major: the slots k
// of all cells are contiguous, so that the first slots of a row of
// neighbouring cells share cache lines (a cell holds about one particle at
// the densities simulated, so a cell-major block of cellcap slots would
// bring a mostly empty line per cell).
__device__ __forceinline__ size_t cell_slot(const Params& P, uint32_t c, uint32_t k) {
    return (size_t)k * P.ncell + c;
}

// Round v * 2^32 to the nearest integer (ties to even) with one FMA: adding
// 1.5 * 2^52 leaves round(v * 2^32) in the low mantissa bits.  Exact for
// |v| < 2^19; larger contributions are clamped and flagged.
__device__ __forceinline__ long long to_fix(double v, uint32_t* err) {
    constexpr double kMagic = 6755399441055744.0;   // 1.5 * 2^52
    if (!(fabs(v) < 524288.0)) {
        atomicOr(err, kErrForce);
        v = v > 0.0 ? 524287.0 : -524287.0;
    }
    return __double_as_longlong(fma(v, 4294967296.0, kMagic)) - __double_as_longlong(kMagic);
}

// 1/x and 1/sqrt(x) in FP64 from the hardware estimates plus two Newton
// steps (relative error ~1e-16; used for forces only, never for decisions).
__device__ __forceinline__ double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// FP32 minimum-image component, used only to discard far candidates before
// the exact FP64 evaluation (its error, ~1e-5, is far below the margins).
__device__ __forceinline__ float mi_delta_f(float xi, float xj, const Params& P) {
    float d = xj - xi;
    if (fabsf(d) > P.halfLf) d -= P.Lf * rintf(d * (1.0f / P.Lf));
    return d;
}

// Position at the last neighbour-list build, kept only for the rebuild test:
// each coordinate as a 21-bit cell index of a grid of spacing L / 2^21 over
// [-L/2, L/2), the three packed into 63 bits (8 bytes instead of 16).
__device__ __forceinline__ uint2 xref_pack(const Params& P, float4 p) {
    auto q = [&](float x) {
        const int v = (int)((x + P.halfLf) * P.xq);
        return (unsigned long long)(v < 0 ? 0 : (v > 0x1FFFFF ? 0x1FFFFF : v));
    };
    const unsigned long long b = q(p.x) | (q(p.y) << 21) | (q(p.z) << 42);
    return make_uint2((uint32_t)b, (uint32_t)(b >> 32));
}

// Has the particle at p moved farther than skin / 2 from its packed build
// position r?  The grid point is the centre of r's grid cell, at most
// sqrt(3) L / 2^22 (plus FP32 rounding) from where the list was built; the
// host takes that off the threshold disp2, so a true displacement beyond
// skin / 2 always triggers (a rebuild may come slightly early, which changes
// nothing computed: the lists only have to contain every pair in range).
__device__ __forceinline__ bool moved_past_skin(const Params& P, uint2 r, float4 p) {
    const unsigned long long b = (unsigned long long)r.x | ((unsigned long long)r.y << 32);
    auto c = [&](unsigned long long v) { return ((float)(v & 0x1FFFFFull) + 0.5f) * P.xqinv - P.halfLf; };
    const float dx = mi_delta_f(c(b), p.x, P), dy = mi_delta_f(c(b >> 21), p.y, P), dz = mi_delta_f(c(b >> 42), p.z, P);
    return dx * dx + dy * dy + dz * dz > P.disp2;
}

// Event counters (attempts, forms, breaks per reaction) are spread over
// kCtrSlots addresses each; a wave adds its total to the slot of its wave
// index, so that the waves of one launch do not queue on one address.  The
// host sums the slots when it reads the counters.
constexpr uint32_t kCtrSlots = 1024;
enum : int { kCtrAttempt = 0, kCtrForm = 1, kCtrBreak = 2 };

__device__ __forceinline__ unsigned long long* ctr_slot(const Dev& D, int a, int kind, uint32_t w) {
    return &D.counters[((size_t)a * 3 + (size_t)kind) * kCtrSlots + (w & (kCtrSlots - 1))];
}

// Append one entry per lane that has `want` set to event list k (0 formed,
// 1 broken): one atomic per wave reserves the wave's run of entries, each
// lane writes at its rank among the wanting lanes.  Valid in divergent code
// (the ballot covers the lanes that reach it).  The order of the entries
// depends on scheduling; the read-out sorts them.
__device__ __forceinline__ void ev_push(const Params& P, const Dev& D, int k, bool want, uint32_t lo, uint32_t hi,
                                        int a) {
    const unsigned long long mask = __ballot(want);
    if (!want) return;
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (rank == 0) base = atomicAdd(&D.evc[k], (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (base + rank < P.evcap[k]) D.ev[k][base + rank] = make_uint2(lo, hi | ((uint32_t)a << 24));
}

__device__ __forceinline__ void count_add(const Dev& D, int a, int kind, uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0 && v) {
        const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        atomicAdd(ctr_slot(D, a, kind, w), (unsigned long long)v);
    }
}

}  // namespace dyb
