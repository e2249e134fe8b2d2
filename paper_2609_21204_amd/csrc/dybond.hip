// Host side of the C ABI declared in include/dybond.h: configuration,
// validation and rate closure (Eqs. epsilon and probs), device memory, kernel
// launches of one time step and of the bonding sweep, graph replay of any
// number of steps (captured step, head, period, span and tail graphs), the
// batched replicas and their autotuner, and the read-out paths.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dybond.h"
#include "kernels.hpp"
#include "batch.hpp"

// Staging array of db_read_bonds_noalloc: the bond table as kNoAllocBonds
// tag pairs followed by kNoAllocBonds bond types (12 MiB).  Each device the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for that
// device (scratch_on), never through the name.
constexpr uint32_t kNoAllocBonds = 1u << 20;
static __device__ __align__(256) uint32_t scratch[3 * kNoAllocBonds];

using namespace dyb;

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kCellCapMin = 16;   // minimum particle slots per cell
thread_local std::string g_create_error;

struct TypeCfg { uint32_t valence = 0; double sigma = 1.0, eps = 1.0, mass = 1.0; };
struct BondCfg { int kind; double k, r0; double lmin = 0, lc1 = 0, lc0 = 0, lmax = 0; };
constexpr uint32_t kAnaHist = 256;              // largest histogram of the network analyses
constexpr uint32_t kAnaWords = kAnaHist + 8;
struct RxRes { double k_on, k_off, eps, p_on, p_off; };
// rate modifier of one reaction: 0 none, 1 melting, 2 slip bond
struct RxMod { int kind = 0; double lam = 0, tm = 0, k_on_m = 0, k_off_m = 0, a = 0; };

struct Timing {
    bool on = false;
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<uint64_t, double>> acc;
};

}  // namespace

// Neighbour-list skin: a smaller skin rebuilds more often but every step
// scans shorter lists; on the 200k gel 37.3 us per step at 0.25 and 0.3,
// 38.2 at 0.4, 39.1 at 0.2 (482.7 vs 495.2 us at 4 M particles, 0.3 vs 0.4).
constexpr double kDefaultSkin = 0.3;

// Steps between spatial renumberings (at the start of a captured span, so a
// multiple of the 120-step span): each costs the sort and a list rebuild,
// and the order decays slowly; 200k gel: 38.4 us per step sorting every 120
// steps, 37.7 every 240, 37.5 every 480 (4 M particles: 504, 492, 494 us).
constexpr uint64_t kSortPeriod = 480;

struct db_system {
    // configuration (host)
    uint32_t n = 0, ntypes = 0;
    double L = 0.0;
    uint32_t seed = 0;
    int device = 0;
    std::vector<TypeCfg> types;
    std::vector<BondCfg> bonds;
    std::vector<db_reaction_desc> rx;
    std::vector<RxMod> mods;               // one per reaction
    std::vector<RxRes> res;
    std::vector<float> pos, vel;
    std::vector<uint32_t> type;
    bool have_particles = false;
    bool vel_given = false;                // false: Maxwell-Boltzmann velocities drawn by validate()
    std::vector<uint32_t> stat_pairs, stat_bt;
    double dt = 0.005, kT = 1.0, gamma = 1.0;
    uint32_t period = 10;
    int kt_source = DB_KT_SETPOINT;
    bool validated = false, committed = false, invalid = false, dead = false;
    std::string err;
    // device state
    Params P{};
    Dev D{};
    std::vector<void*> allocs;
    hipStream_t stream = nullptr, own_stream = nullptr;
    uint32_t* bsum = nullptr;       // block sums for the bond read-out (nb + 1)
    float4* stage = nullptr;        // tag-ordered staging buffer
    uint32_t* flag = nullptr;       // device flag for iterative kernels
    uint32_t* err_h = nullptr;      // pinned host copy of the device error words
    uint64_t step = 0;
    int cur_x = 0, cur_list = 0;
    std::vector<uint32_t> tag_h, rtag_h;   // host mirrors of tag / rtag
    std::vector<PairTab> pair_h;           // WCA table uploaded to D.pair
    Timing timing;
    std::map<uint64_t, hipGraphExec_t> graphs;   // captured step graphs, by kind and phase (graph_key)
    hipEvent_t ev_out = nullptr, ev_back = nullptr;   // ordering of device-side read-outs
    uint32_t* bref = nullptr;              // reference bond table of the bond correlation (by tag)
    bool have_ref = false;
    unsigned long long* ana = nullptr;     // analysis results (device, kAnaWords words)
    bool use_graphs = true;
    uint32_t cellcap_user = 0;             // 0 = automatic
    double skin = kDefaultSkin;            // neighbour-list skin
    uint32_t nlmax_user = 0;               // neighbour-list slots per particle, 0 = automatic
    uint32_t tpp_user = 0;                 // threads per particle in k_step and k_propose, 0 = automatic
    uint32_t qb_user = 0;                  // list entries per thread issued up front in k_step, 0 = automatic
    uint32_t match_rounds = 1;             // full-grid matching rounds before the one-workgroup finish
    uint32_t finish_lds = kFinishLds;      // largest live list the finish matches in LDS
    bool tags_dirty = false;               // device tag/rtag changed since the host mirrors were read
    bool sort_enabled = true;              // renumber particles in cell order (every kSortPeriod steps)
    uint64_t sort_due = 0;                 // step from which the next renumbering is due
    int path_pick = 0;                     // long calls on a small system: 0 not measured, 1 one workgroup, 2 grid
    bool path_pending = false;             // a measurement of the two paths awaits the end of the call
    hipEvent_t path_ev[3] = {nullptr, nullptr, nullptr};
};

namespace {

db_status fail(db_system* s, db_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_create_error = buf;
    return st;
}

#define HIPCHK(sys, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (sys)->dead = true;                                                                  \
            return fail((sys), DB_EDEVICE, "HIP error %s at %s:%d", hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                                     \
        }                                                                                        \
    } while (0)

inline unsigned grid_of(uint32_t n) { return (n + kBlock - 1) / kBlock; }
inline unsigned ntiles(const Params& P) { return P.ntile[0] * P.ntile[1] * P.ntile[2]; }


struct TimerScope {
    db_system* s;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    TimerScope(db_system* sys, const char* nm) : s(sys), name(nm) {
        if (!s->timing.on) return;
        auto take = [&]() {
            hipEvent_t e;
            if (!s->timing.pool.empty()) { e = s->timing.pool.back(); s->timing.pool.pop_back(); }
            else (void)hipEventCreate(&e);
            return e;
        };
        a = take();
        b = take();
    }
    ~TimerScope() {
        if (!a) return;
        std::string nm(name);
        const size_t lt = nm.find('<');      // k_step<4> is reported as k_step
        if (lt != std::string::npos) nm.resize(lt);
        s->timing.pending.push_back({nm, a, b});
    }
};

// With timing on, the launch carries a start and a stop event that the
// runtime stamps when the kernel itself begins and ends (not when the stream
// reaches the launch), so the per-kernel times are kernel execution times.
#define LAUNCH(sys, kern, grid, block, ...) LAUNCH_AS(sys, #kern, kern, grid, block, __VA_ARGS__)
// kernels built in two variants: the full one for systems with tether bonds
// or rate modifiers, the lean one otherwise
#define LAUNCH_EXT(sys, tname, kern, grid, block, ...)                                       \
    do {                                                                                     \
        if ((sys)->P.ext) LAUNCH_AS(sys, tname, (kern<true>), grid, block, __VA_ARGS__);     \
        else LAUNCH_AS(sys, tname, (kern<false>), grid, block, __VA_ARGS__);                 \
    } while (0)
// the same, with the name the kernel is timed under given explicitly
#define LAUNCH_AS(sys, tname, kern, grid, block, ...)                                            \
    do {                                                                                         \
        TimerScope ts_((sys), tname);                                                            \
        if (ts_.a)                                                                               \
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (sys)->stream, ts_.a, ts_.b, \
                                  0u, __VA_ARGS__);                                              \
        else                                                                                     \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (sys)->stream, __VA_ARGS__);   \
    } while (0)

void flush_timing(db_system* s) {
    if (s->timing.pending.empty()) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto& p : s->timing.pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        auto& acc = s->timing.acc[p.name];
        acc.first += 1;
        acc.second += ms;
        s->timing.pool.push_back(p.a);
        s->timing.pool.push_back(p.b);
    }
    s->timing.pending.clear();
}

bool isnan_(double v) { return std::isnan(v); }

// Rate closure of one reaction (Eq. epsilon: K = k_on/k_off = e^eps; Eq. probs:
// P0 = k n dt).  Same order of evaluation as documented in the header.
db_status close_rates(db_system* s, const db_reaction_desc& d, RxRes& out) {
    double k_on = d.k_on, k_off = d.k_off, eps = d.epsilon, p_on0 = d.p_on0;
    const double ndt = (double)s->period * s->dt;
    if (!isnan_(p_on0)) {
        if (!isnan_(k_on)) {
            if (std::fabs(p_on0 - k_on * ndt) > 1e-9 * std::max(1.0, std::fabs(p_on0)))
                return fail(s, DB_EINVAL, "reaction: k_on and p_on0 disagree");
        } else {
            k_on = p_on0 / ndt;
        }
    }
    const int known = !isnan_(k_on) + !isnan_(k_off) + !isnan_(eps);
    if (known < 2) return fail(s, DB_EINVAL, "reaction: rates under-determined (give two of k_on/p_on0, k_off, epsilon)");
    if (!isnan_(k_on) && !isnan_(k_off)) {
        if (!isnan_(eps)) {
            if (k_off <= 0.0 || k_on <= 0.0 ||
                std::fabs(eps - std::log(k_on / k_off)) > 1e-9 * std::max(1.0, std::fabs(eps)))
                return fail(s, DB_EINVAL, "reaction: k_on, k_off and epsilon disagree");
        } else if (k_on > 0.0 && k_off > 0.0) {
            eps = std::log(k_on / k_off);
        }
    } else if (!isnan_(k_on)) {
        k_off = k_on * std::exp(-eps);
    } else {
        k_on = k_off * std::exp(eps);
    }
    const double p_on = !isnan_(p_on0) ? p_on0 : k_on * ndt;
    const double p_off = k_off * ndt;
    for (double v : {k_on, k_off, p_on, p_off})
        if (!std::isfinite(v) || v < 0.0) return fail(s, DB_ERANGE, "reaction: negative or non-finite rate");
    if (p_on > 1.0 || p_off > 1.0)
        return fail(s, DB_ERANGE, "reaction: per-sweep probability k n dt exceeds 1 (P0_on=%g, P0_off=%g)", p_on, p_off);
    out = RxRes{k_on, k_off, eps, p_on, p_off};
    return DB_OK;
}

double wca_cut(double sig) { return std::pow(2.0, 1.0 / 6.0) * sig; }

// The requested skin, shrunk so that the box still holds 3 cells of side
// r_search + skin (negative when even skin 0 does not fit).
double effective_skin(const db_system* s, double rsearch) {
    const double room = s->L / (3.0 * (1.0 + 1e-5)) - rsearch;
    return std::min(s->skin, room);
}

// Velocities of the set-point temperature kT with zero total momentum, for a
// db_set_particles call without velocities: component c of tag t is
// sqrt(kT / m) g_c with three standard normals g from Box-Muller on the block
// (0, 0, t, 0) of the INIT stream (u1 = (w + 1) / 2^32 in (0, 1],
// u2 = w' / 2^32), then the mass-weighted mean velocity is subtracted.
void draw_velocities(db_system* s) {
    const uint32_t n = s->n;
    std::vector<double> v(3 * (size_t)n);
    double px = 0.0, py = 0.0, pz = 0.0, msum = 0.0;
    const uint32_t k1 = stream_k1(kInit, 0, 0);
    const double twopi = 2.0 * 3.14159265358979323846;
    for (uint32_t t = 0; t < n; ++t) {
        const Word4 w = philox(0u, 0u, t, 0u, s->seed, k1);
        const double ra = std::sqrt(-2.0 * std::log(((double)w.w0 + 1.0) * 0x1.0p-32));
        const double ta = twopi * ((double)w.w1 * 0x1.0p-32);
        const double rb = std::sqrt(-2.0 * std::log(((double)w.w2 + 1.0) * 0x1.0p-32));
        const double tb = twopi * ((double)w.w3 * 0x1.0p-32);
        const double m = s->types[s->type[t]].mass, sd = std::sqrt(s->kT / m);
        v[3 * (size_t)t] = sd * (ra * std::cos(ta));
        v[3 * (size_t)t + 1] = sd * (ra * std::sin(ta));
        v[3 * (size_t)t + 2] = sd * (rb * std::cos(tb));
        px += m * v[3 * (size_t)t];
        py += m * v[3 * (size_t)t + 1];
        pz += m * v[3 * (size_t)t + 2];
        msum += m;
    }
    s->vel.resize(3 * (size_t)n);
    for (uint32_t t = 0; t < n; ++t) {
        s->vel[3 * (size_t)t] = (float)(v[3 * (size_t)t] - px / msum);
        s->vel[3 * (size_t)t + 1] = (float)(v[3 * (size_t)t + 1] - py / msum);
        s->vel[3 * (size_t)t + 2] = (float)(v[3 * (size_t)t + 2] - pz / msum);
    }
}

db_status validate(db_system* s) {
    s->validated = false;
    if (!s->have_particles) return fail(s, DB_ESTATE, "particles not set");
    if (!(s->dt > 0.0) || !(s->kT >= 0.0) || !(s->gamma >= 0.0) || s->period < 1)
        return fail(s, DB_EINVAL, "integrator parameters out of range");
    if (s->rx.size() > (size_t)kMaxRx) return fail(s, DB_EINVAL, "too many reactions");
    s->res.assign(s->rx.size(), RxRes{});
    std::vector<int> bt_owner(s->bonds.size(), -1);
    double rmax_all = 0.0;
    for (size_t a = 0; a < s->rx.size(); ++a) {
        const auto& d = s->rx[a];
        if (d.self_avoid != 0 && d.self_avoid != 1)
            return fail(s, DB_EINVAL, "reaction %zu: self_avoid must be stated as 0 or 1", a);
        if (d.type_a >= s->ntypes || d.type_b >= s->ntypes)
            return fail(s, DB_EINVAL, "reaction %zu: type out of range", a);
        if (d.bond_type >= s->bonds.size()) return fail(s, DB_EINVAL, "reaction %zu: bond type out of range", a);
        const BondCfg& bc = s->bonds[d.bond_type];
        if (bc.kind == DB_BOND_FENE && !(d.r_max < bc.r0))
            return fail(s, DB_EINVAL, "reaction %zu: a FENE reaction window must end below R0", a);
        if (bc.kind == DB_BOND_TETHER && !(bc.lmin < d.r_min && d.r_max < bc.lmax))
            return fail(s, DB_EINVAL, "reaction %zu: a tether reaction window must lie inside (l_min, l_max)", a);
        if (bt_owner[d.bond_type] >= 0)
            return fail(s, DB_EINVAL, "reaction %zu: bond type already owned by reaction %d", a, bt_owner[d.bond_type]);
        bt_owner[d.bond_type] = (int)a;
        if (!(d.r_min >= 0.0) || !(d.r_max > d.r_min) || !std::isfinite(d.r_max))
            return fail(s, DB_EINVAL, "reaction %zu: window must satisfy 0 <= r_min < r_max", a);
        rmax_all = std::max(rmax_all, d.r_max);
        db_status st = close_rates(s, d, s->res[a]);
        if (st != DB_OK) return st;
        const RxMod& m = s->mods[a];
        if (m.kind == 1) {
            const double ndt = (double)s->period * s->dt;
            const double pm_on = m.k_on_m * ndt, pm_off = m.k_off_m * ndt;
            if (!(pm_on >= 0.0 && pm_on <= 1.0 && pm_off >= 0.0 && pm_off <= 1.0))
                return fail(s, DB_ERANGE, "reaction %zu: melted rate k n dt outside [0, 1]", a);
        }
    }
    for (const auto& b : s->bonds)
        if (b.kind != DB_BOND_TETHER && (!(b.k >= 0.0) || !(b.r0 > 0.0 || (b.kind == DB_BOND_HARMONIC && b.r0 >= 0.0))))
            return fail(s, DB_EINVAL, "bond type parameters out of range");
    double rc = 0.0;
    for (uint32_t a = 0; a < s->ntypes; ++a)
        for (uint32_t b = 0; b < s->ntypes; ++b) {
            const double sig = 0.5 * (s->types[a].sigma + s->types[b].sigma);
            const double eps = std::sqrt(s->types[a].eps * s->types[b].eps);
            if (sig > 0.0 && eps > 0.0) rc = std::max(rc, wca_cut(sig));
        }
    const double rsearch = std::max(rc, rmax_all);
    if (!(rsearch > 0.0)) return fail(s, DB_EINVAL, "no interaction range (all sigma 0 and no reaction)");
    if (effective_skin(s, rsearch) < 0.0)
        return fail(s, DB_EINVAL, "box L=%g holds fewer than 3 cells of side %g", s->L, rsearch);
    const double nc = std::floor(s->L / ((rsearch + effective_skin(s, rsearch)) * (1.0 + 1e-5)));
    if (nc * nc * nc > 2.0e9) return fail(s, DB_EINVAL, "too many cells");
    // static bonds: per particle degree, FENE range
    std::vector<uint32_t> deg(s->n, 0);
    for (size_t k = 0; k < s->stat_bt.size(); ++k) {
        const uint32_t i = s->stat_pairs[2 * k], j = s->stat_pairs[2 * k + 1];
        if (i >= s->n || j >= s->n || i == j || s->stat_bt[k] >= s->bonds.size())
            return fail(s, DB_EINVAL, "static bond %zu invalid", k);
        if (++deg[i] > (uint32_t)kMaxStatic || ++deg[j] > (uint32_t)kMaxStatic)
            return fail(s, DB_EINVAL, "more than %d static bonds on one particle", kMaxStatic);
    }
    if (!s->vel_given) draw_velocities(s);
    s->validated = true;
    return DB_OK;
}

void union_find_mol(db_system* s, std::vector<uint32_t>& mol) {
    mol.resize(s->n);
    std::iota(mol.begin(), mol.end(), 0u);
    auto find = [&](uint32_t v) {
        while (mol[v] != v) { mol[v] = mol[mol[v]]; v = mol[v]; }
        return v;
    };
    for (size_t k = 0; k < s->stat_bt.size(); ++k) {
        uint32_t a = find(s->stat_pairs[2 * k]), b = find(s->stat_pairs[2 * k + 1]);
        if (a != b) mol[std::max(a, b)] = std::min(a, b);
    }
    for (uint32_t v = 0; v < s->n; ++v) mol[v] = find(v);
}

template <class T>
db_status dalloc(db_system* s, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(s, DB_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    s->allocs.push_back(q);
    *p = (T*)q;
    return DB_OK;
}

#define DALLOC(sys, ptr, count)                       \
    do {                                              \
        db_status st_ = dalloc((sys), &(ptr), (count)); \
        if (st_ != DB_OK) return st_;                 \
    } while (0)

// Slots per cell: room for a Poisson fluctuation far above the mean occupancy
// and at least twice the fullest cell of the state being uploaded.
uint32_t cell_capacity(const db_system* s, const Params& P, const float* pos3 = nullptr) {
    if (s->cellcap_user) return s->cellcap_user;
    const double lam = (double)s->n / (double)P.ncell;
    double cap = lam + 8.0 * std::sqrt(lam) + 8.0;
    const float* x = pos3 ? pos3 : s->pos.data();
    if (x) {
        std::vector<uint32_t> occ(P.ncell, 0);
        uint32_t mx = 0;
        auto cc = [&](float v) {
            int c = (int)std::floor((v + P.halfLf) * P.cell_scale);
            return std::min(std::max(c, 0), (int)P.nc - 1);
        };
        for (uint32_t i = 0; i < s->n; ++i) {
            const size_t c = ((size_t)cc(x[3 * i + 2]) * P.nc + cc(x[3 * i + 1])) * P.nc + cc(x[3 * i]);
            mx = std::max(mx, ++occ[c]);
        }
        cap = std::max(cap, 2.0 * mx);
    }
    uint32_t c = std::max<uint32_t>(kCellCapMin, (uint32_t)std::ceil(cap));
    return (c + 7u) & ~7u;
}

// Cells per neighbour-list tile (t x t x t): the widest tile whose halo,
// (t + 2)^3 cells, fits the LDS tables (at most kTileMaxHalo cells, on
// average at most 3/4 of kTileMaxEntries particles so that clusters denser
// than the mean still fit) and that still leaves at least 512 tiles to cover
// the chip; the narrowest admissible tile when no width gives 512.
void choose_tiles(const db_system* s, Params& P) {
    const double lam = std::max((double)s->n / (double)P.ncell, 1e-6);
    auto ntiles_of = [&](int tt) {
        const long k = ((long)P.nc + tt - 1) / tt;
        return k * k * k;
    };
    int t = 1;
    for (int tt = std::min(10, (int)P.nc); tt >= 1; --tt) {
        const double halo = (double)(tt + 2) * (tt + 2) * (tt + 2);
        if (halo > kTileMaxHalo || lam * halo > 0.75 * kTileMaxEntries) continue;
        t = tt;
        if (ntiles_of(tt) >= 512) break;
    }
    for (int d = 0; d < 3; ++d) {
        P.tile[d] = (uint32_t)t;
        P.ntile[d] = (P.nc + (uint32_t)t - 1) / (uint32_t)t;
    }
}

// The cells of an nc^3 grid (index (z nc + y) nc + x) in Morton order: sorted
// by the interleaved bits of (x, y, z), x in the lowest bit of each triple.
std::vector<uint32_t> morton_cells(uint32_t nc) {
    auto spread = [](uint64_t v) {          // bit b of v moves to bit 3b
        uint64_t r = 0;
        for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
        return r;
    };
    std::vector<uint64_t> sx(nc), sy(nc), sz(nc);
    for (uint32_t k = 0; k < nc; ++k) {
        sx[k] = spread(k);
        sy[k] = spread(k) << 1;
        sz[k] = spread(k) << 2;
    }
    const uint64_t ncell = (uint64_t)nc * nc * nc;
    std::vector<uint64_t> key(ncell);     // Morton code (< 2^33 for nc < 2048) above the cell index
    for (uint64_t c = 0; c < ncell; ++c) {
        const uint64_t x = c % nc, y = (c / nc) % nc, z = c / ((uint64_t)nc * nc);
        key[c] = ((sx[x] | sy[y] | sz[z]) << 31) | c;
    }
    std::sort(key.begin(), key.end());
    std::vector<uint32_t> out(ncell);
    for (uint64_t r = 0; r < ncell; ++r) out[r] = (uint32_t)(key[r] & 0x7FFFFFFFull);
    return out;
}

// Melting modifier at temperature T (Eqs. gT, kT): P = P_init (1 - g) + P_melt g,
// g = [tanh(lambda (T - T_melt)) + 1] / 2; P0 = k n dt is linear in k.
double melt_mix_host(double p_init, double p_melt, double lam, double tm, double T) {
#pragma clang fp contract(off)
    const double g = 0.5 * (tanh_det(lam * (T - tm)) + 1.0);
    return p_init * (1.0 - g) + p_melt * g;
}

// Step tables: the same numbers k_step would read from the parameter block,
// laid out for one 16-byte copy per thread into LDS.
void fill_tabs(const db_system* s, StepTabs& th) {
    const Params& P = s->P;
    th = StepTabs{};
    for (int k = 0; k < kMaxTypes * kMaxTypes; ++k) {
        th.rc2_pre[k] = P.rc2_pre[k];
        th.rc2_in[k] = P.rc2_in[k];
        th.sig2f[k] = P.sig2f[k];
        th.eps24f[k] = P.eps24f[k];
        th.rl2[k] = P.rl2[k];
        th.pair[k] = s->pair_h[k];
    }
    for (int k = 0; k < 8; ++k) {
        th.bk[k] = P.bk[k];
        th.br0[k] = P.br0[k];
        th.binvR02[k] = P.binvR02[k];
        th.blmin[k] = P.blmin[k];
        th.blc1[k] = P.blc1[k];
        th.blc0[k] = P.blc0[k];
        th.blmax[k] = P.blmax[k];
        th.bkind[k] = P.bkind[k];
        th.rbt[k] = P.rbt[k];
        th.hm[k] = P.h * P.inv_mass[k];
        th.noise_sd[k] = P.noise_sd[k];
        th.mass[k] = P.mass[k];
        th.cap[k] = P.cap[k];
    }
}

// The parts of the parameters that depend on the temperature: the noise
// amplitudes and, at a set-point temperature, the melted probabilities.
void apply_temperature(db_system* s) {
    Params& P = s->P;
    const double c1 = std::exp(-s->gamma * s->dt);
    P.kT = s->kT;
    for (uint32_t t = 0; t < s->ntypes; ++t)
        P.noise_sd[t] = (float)(std::sqrt(std::max(0.0, 1.0 - c1 * c1)) * std::sqrt(s->kT / s->types[t].mass));
    for (size_t a = 0; a < s->rx.size(); ++a)
        if (s->mods[a].kind == 1 && s->kt_source != DB_KT_KINETIC) {
            P.pon[a] = melt_mix_host(P.pon_i[a], P.pon_m[a], P.mlam[a], P.mtm[a], s->kT);
            P.poff[a] = melt_mix_host(P.poff_i[a], P.poff_m[a], P.mlam[a], P.mtm[a], s->kT);
        }
}

// Automatic launch shapes (threads per particle) of the step kernel and of
// the proposal kernel, measured on the gel and the sweep replicas (µs per
// step, shapes given as step / proposal threads):
//  - below 32 768 particles 8 / 8: 10 500 particles 13.4 against 14.1 at
//    4 / 4 and 18.0 at 32 / 16 (the earlier rule of at least 2^19 threads
//    per launch), 20 000 particles 17.8 against 18.7 and 26.2;
//  - up to 1.5 M particles 4 / 2: 50 000 particles 21.7 against 22.0 at
//    8 / 8, 200 000 particles 35.9 against 40.3;
//  - from 1.5 M particles on 1 / 2: once the state no longer sits in the
//    Infinity Cache, one thread per particle (k_step1, whose loads for a
//    particle are all in flight together and which needs no LDS reduction)
//    beats four: 2 M particles 3.7 % faster per step, 4 M 6.6 %, 16 M 7.9 %
//    (equal at 1 M).
constexpr uint32_t kStepEightThreadN = 32768u, kStepOneThreadN = 1500000u;
uint32_t auto_step_tpp(uint32_t n) { return n >= kStepOneThreadN ? 1u : (n < kStepEightThreadN ? 8u : 4u); }
uint32_t auto_propose_tpp(uint32_t n) { return n < kStepEightThreadN ? 8u : 2u; }

void fill_params(db_system* s) {
    Params& P = s->P;
    P = Params{};
    P.n = s->n;
    P.ntypes = s->ntypes;
    P.nrx = (uint32_t)s->rx.size();
    P.seed = s->seed;
    P.period = s->period;
    P.kt_kinetic = s->kt_source == DB_KT_KINETIC;
    P.L = s->L;
    P.invL = 1.0 / s->L;
    P.Lf = (float)s->L;
    P.halfLf = (float)(0.5 * s->L);
    P.h = (float)(0.5 * s->dt);
    const double c1 = std::exp(-s->gamma * s->dt);
    P.c1 = (float)c1;
    P.kT = s->kT;
    uint32_t capmax = 0;
    for (uint32_t t = 0; t < s->ntypes; ++t) {
        P.inv_mass[t] = (float)(1.0 / s->types[t].mass);
        P.mass[t] = (float)s->types[t].mass;
        P.noise_sd[t] = (float)(std::sqrt(std::max(0.0, 1.0 - c1 * c1)) * std::sqrt(s->kT / s->types[t].mass));
        P.cap[t] = s->types[t].valence;
        capmax = std::max(capmax, s->types[t].valence);
    }
    P.cap_max = std::max(capmax, 1u);
    double rc = 0.0, rmax_all = 0.0;
    s->pair_h.assign(kMaxTypes * kMaxTypes, PairTab{0.0, 0.0, 0.0, -1.0, -1.0, 0.0, 0.0, 0.0});
    for (uint32_t a = 0; a < s->ntypes; ++a)
        for (uint32_t b = 0; b < s->ntypes; ++b) {
            const double sig = 0.5 * (s->types[a].sigma + s->types[b].sigma);
            const double eps = std::sqrt(s->types[a].eps * s->types[b].eps);
            const int k = a * kMaxTypes + b;
            if (sig > 0.0 && eps > 0.0) {
                const double c = wca_cut(sig);
                s->pair_h[k] = PairTab{sig * sig, 24.0 * eps, c, c * c * (1.0 - 1e-14), c * c * (1.0 + 1e-14),
                                       eps, 0.0, 0.0};
                P.rc2_pre[k] = (float)(c * c * (1.0 + 1e-3) + 1e-4);
                P.rc2_in[k] = (float)(0.98 * 0.98 * c * c);
                P.sig2f[k] = (float)(sig * sig);
                P.eps24f[k] = (float)(24.0 * eps);
                rc = std::max(rc, c);
            }
        }
    for (size_t b = 0; b < s->bonds.size(); ++b) {
        P.bkind[b] = (uint32_t)s->bonds[b].kind;
        P.bk[b] = s->bonds[b].k;
        P.br0[b] = s->bonds[b].r0;
        P.bR02[b] = s->bonds[b].r0 * s->bonds[b].r0;
        P.binvR02[b] = P.bR02[b] > 0.0 ? 1.0 / P.bR02[b] : 0.0;
        P.blmin[b] = s->bonds[b].lmin;
        P.blc1[b] = s->bonds[b].lc1;
        P.blc0[b] = s->bonds[b].lc0;
        P.blmax[b] = s->bonds[b].lmax;
        if (s->bonds[b].kind == DB_BOND_TETHER) P.ext = 1u;
    }
    for (size_t a = 0; a < s->rx.size(); ++a) {
        const auto& d = s->rx[a];
        P.ra[a] = d.type_a;
        P.rb[a] = d.type_b;
        P.rbt[a] = d.bond_type;
        P.rself[a] = (uint32_t)d.self_avoid;
        P.any_self_avoid |= (uint32_t)d.self_avoid;
        P.rmin[a] = d.r_min;
        P.rmax[a] = d.r_max;
        // target length of proposals: the minimum of the reaction's bond
        // potential (harmonic r0, FENE 0, tether the middle of its flat region)
        const BondCfg& bc = s->bonds[d.bond_type];
        P.r0[a] = bc.kind == DB_BOND_FENE ? 0.0 : bc.r0;
        P.hk[a] = 0.5 * bc.k;
        P.pon[a] = s->res[a].p_on;
        P.poff[a] = s->res[a].p_off;
        const RxMod& m = s->mods[a];
        if (m.kind != 0 || bc.kind != DB_BOND_HARMONIC) P.ext = 1u;
        P.rmod[a] = (uint32_t)m.kind;
        P.slip[a] = m.a;
        if (m.kind == 1) {
            const double ndt = (double)s->period * s->dt;
            P.mlam[a] = m.lam;
            P.mtm[a] = m.tm;
            P.pon_i[a] = s->res[a].p_on;
            P.poff_i[a] = s->res[a].p_off;
            P.pon_m[a] = m.k_on_m * ndt;
            P.poff_m[a] = m.k_off_m * ndt;
            if (s->kt_source != DB_KT_KINETIC) {      // fixed temperature: mix once here
                P.pon[a] = melt_mix_host(P.pon_i[a], P.pon_m[a], m.lam, m.tm, s->kT);
                P.poff[a] = melt_mix_host(P.poff_i[a], P.poff_m[a], m.lam, m.tm, s->kT);
            }
        }
        P.rmax2_pre[a] = (float)(d.r_max * d.r_max * (1.0 + 1e-3) + 1e-4);
        P.rmin2_pre[a] = (float)std::max(0.0, d.r_min * d.r_min * (1.0 - 1e-3) - 1e-4);
        rmax_all = std::max(rmax_all, d.r_max);
    }
    const double rsearch = std::max(rc, rmax_all);
    const double skin = effective_skin(s, rsearch);
    const double rlist = rsearch + skin;
    // list radius per type pair: the WCA cutoff or the largest r_max of a
    // reaction between the two types, plus the skin
    for (uint32_t a = 0; a < s->ntypes; ++a)
        for (uint32_t b = 0; b < s->ntypes; ++b) {
            double need = s->pair_h.empty() ? 0.0 : s->pair_h[a * kMaxTypes + b].rc;
            for (const auto& d : s->rx)
                if ((d.type_a == a && d.type_b == b) || (d.type_a == b && d.type_b == a)) need = std::max(need, d.r_max);
            const double rl = need > 0.0 ? need + skin : 0.0;
            P.rl2[a * kMaxTypes + b] = (float)(rl * rl * (1.0 + 1e-4));
        }
    // from 32 768 particles on, the proposal kernel takes 2 threads per site
    // by default: its scan is shorter (4 list entries up front) and its
    // listed sites more numerous per pass (13.3 vs 15.9 us per reaction at
    // 200k particles with 2 vs 4 threads, 145 vs 168 us at 4 M); below, 8
    // like the step kernel (auto_propose_tpp)
    P.tpp_step = s->tpp_user ? s->tpp_user : auto_step_tpp(s->n);
    P.tpp = s->tpp_user ? s->tpp_user : auto_propose_tpp(s->n);
    P.qb_step = P.tpp_step == 4 ? s->qb_user : 0u;
    // build positions are packed to a 21-bit grid (xref_pack): the test takes
    // the grid's half spacing and the FP32 rounding of its decoding off skin / 2
    P.xq = (float)(2097152.0 / s->L);
    P.xqinv = (float)(s->L / 2097152.0);
    const double qerr = std::sqrt(3.0) * (s->L / 4194304.0 + s->L * 0x1.0p-22) * 1.01;
    const double thr = std::max(0.0, 0.5 * skin - 1e-4 - qerr);
    P.disp2 = (float)(thr * thr);
    // neighbour slots: room for 2.5x the mean count of an ideal gas at this
    // density plus 32, at least 64 (or exactly what the caller asked for)
    const double mean_nb = 4.18879020478639 * rlist * rlist * rlist * (double)s->n / (s->L * s->L * s->L);
    const uint32_t auto_nl = (std::max<uint32_t>(64u, (uint32_t)std::ceil(2.5 * mean_nb + 32.0)) + 7u) & ~7u;
    P.nlmax = s->nlmax_user ? s->nlmax_user : auto_nl;

    P.nc = (uint32_t)std::floor(s->L / (rlist * (1.0 + 1e-5)));
    P.ncell = P.nc * P.nc * P.nc;
    P.cell_scale = (float)((double)P.nc / s->L);
    P.cellcap = cell_capacity(s, P);
    choose_tiles(s, P);
    uint32_t smax = 0;
    std::vector<uint32_t> deg(s->n, 0);
    for (size_t k = 0; k < s->stat_bt.size(); ++k) {
        smax = std::max(smax, ++deg[s->stat_pairs[2 * k]]);
        smax = std::max(smax, ++deg[s->stat_pairs[2 * k + 1]]);
    }
    P.stat_max = smax;
}

// Upload positions/velocities (tag order) and dynamic bonds; rebuild derived
// device state (cell list, u = v - h F/m).  With `vel_is_u` the velocities
// are already the integrator's carried velocity u (a checkpoint), stored as
// given; img3 (tag order, NULL = zeros) sets the periodic image counters.
db_status upload_state(db_system* s, const float* pos3, const float* vel3, const uint32_t* pairs,
                       const uint32_t* bts, uint64_t m, bool vel_is_u = false, const int32_t* img3 = nullptr) {
    const uint32_t n = s->n;
    if (s->tags_dirty) {
        HIPCHK(s, hipMemcpyAsync(s->tag_h.data(), s->D.tag, n * 4, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipMemcpyAsync(s->rtag_h.data(), s->D.rtag, n * 4, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        s->tags_dirty = false;
    }
    const Params& P = s->P;
    std::vector<float4> xs(n), vs(n);
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t t = s->tag_h[i];
        float tb;
        const uint32_t ty = s->type[t];
        std::memcpy(&tb, &ty, 4);
        xs[i] = make_float4(pos3[3 * t], pos3[3 * t + 1], pos3[3 * t + 2], tb);
        float tg;                          // the tag rides in u's w word
        std::memcpy(&tg, &t, 4);
        vs[i] = make_float4(vel3[3 * t], vel3[3 * t + 1], vel3[3 * t + 2], tg);
    }
    std::vector<uint32_t> dyn((size_t)P.cap_max * n, kEmpty);
    std::vector<uint8_t> occ(n, 0);
    std::vector<int> bt2rx(s->bonds.size(), -1);
    for (size_t a = 0; a < s->rx.size(); ++a) bt2rx[s->rx[a].bond_type] = (int)a;
    for (uint64_t k = 0; k < m; ++k) {
        const uint32_t ta = pairs[2 * k], tb = pairs[2 * k + 1], bt = bts[k];
        const int a = bt < bt2rx.size() ? bt2rx[bt] : -1;
        const uint32_t ia = s->rtag_h[ta], ib = s->rtag_h[tb];
        const uint32_t bits = ((uint32_t)a << 24);
        auto put = [&](uint32_t i, uint32_t j) {
            for (uint32_t q = 0; q < P.cap_max; ++q)
                if (dyn[(size_t)q * n + i] == kEmpty) { dyn[(size_t)q * n + i] = j | bits; return; }
        };
        put(ia, ib);
        put(ib, ia);
        occ[ia]++;
        occ[ib]++;
    }
    std::vector<int32_t> img(3 * (size_t)n, 0);
    if (img3)
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t d = 0; d < 3; ++d) img[(size_t)d * n + i] = img3[3 * (size_t)s->tag_h[i] + d];
    HIPCHK(s, hipMemcpyAsync(s->D.x[0], xs.data(), n * sizeof(float4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D.x[1], xs.data(), n * sizeof(float4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D.u, vs.data(), n * sizeof(float4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D.dyn, dyn.data(), dyn.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D.occ, occ.data(), n, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D.img, img.data(), img.size() * 4, hipMemcpyHostToDevice, s->stream));
    unsigned long long sv[2];
    sv[s->step & 1] = s->step;
    sv[(s->step & 1) ^ 1] = s->step;
    HIPCHK(s, hipMemcpyAsync(s->D.stepv, sv, sizeof sv, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(s->D.err, 0, 4 * sizeof(uint32_t), s->stream));
    HIPCHK(s, hipMemsetAsync(s->D.ke_fix, 0, 2 * sizeof(unsigned long long), s->stream));
    // no sweep has run on this state yet: empty event lists, step key all ones
    const uint32_t evc0[4] = {0u, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu};
    HIPCHK(s, hipMemcpyAsync(s->D.evc, evc0, sizeof evc0, hipMemcpyHostToDevice, s->stream));
    // lists built below, from cell list 0 (all three cleared)
    const uint32_t flags[4] = {s->step % 3 == 0, s->step % 3 == 1, s->step % 3 == 2, 0u};
    HIPCHK(s, hipMemcpyAsync(s->D.rflag, flags, sizeof flags, hipMemcpyHostToDevice, s->stream));
    s->cur_x = (int)(s->step & 1u);        // buffer indices follow the step counter
    s->cur_list = (int)(s->step % 3);
    s->sort_due = s->step;                 // uploaded in tag order: renumber at the next period boundary
    for (int l = 0; l < 3; ++l) LAUNCH(s, k_clear_counts, std::min(grid_of(P.ncell), 65535u), kBlock, s->P, s->D, l);
    LAUNCH(s, k_binr, grid_of(n), kBlock, s->P, s->D, s->cur_x, (int)(s->step % 3));
    LAUNCH(s, k_nlist, ntiles(P), kTileThreads, s->P, s->D, (int)(s->step % 3));
    LAUNCH(s, k_eval, grid_of(n), kBlock, s->P, s->D, s->cur_x, 0u);
    if (!vel_is_u) LAUNCH(s, k_init_u, grid_of(n), kBlock, s->P, s->D, s->cur_x, 0u);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipStreamSynchronize(s->stream));
    uint32_t err[4];
    HIPCHK(s, hipMemcpy(err, s->D.err, sizeof err, hipMemcpyDeviceToHost));
    if (err[0] & kErrOverflow) { s->invalid = true; return fail(s, DB_EOVERFLOW, "cell capacity %u exceeded", s->P.cellcap); }
    if (err[0] & kErrFene) { s->invalid = true; return fail(s, DB_EBOND, "bond %u-%u outside its range (FENE r >= R0, tether r outside (l_min, l_max))", err[1], err[2]); }
    if (err[0] & kErrForce) { s->invalid = true; return fail(s, DB_EBOND, "force out of range"); }
    if (err[0] & kErrNlist) { s->invalid = true; return fail(s, DB_EOVERFLOW, "more than %u neighbours of one particle", s->P.nlmax); }
    s->invalid = false;
    return DB_OK;
}

void destroy_graphs(db_system* s) {
    for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
    s->graphs.clear();
}

// Grow the per-cell member arrays when a new state needs more slots per cell.
db_status ensure_cell_capacity(db_system* s, const float* pos3) {
    const uint32_t need = cell_capacity(s, s->P, pos3);
    if (need <= s->P.cellcap) return DB_OK;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int l = 0; l < 3; ++l) {
        auto it = std::find(s->allocs.begin(), s->allocs.end(), (void*)s->D.cpos[l]);
        if (it != s->allocs.end()) s->allocs.erase(it);
        HIPCHK(s, hipFree(s->D.cpos[l]));
        s->D.cpos[l] = nullptr;
        DALLOC(s, s->D.cpos[l], (size_t)s->P.ncell * need);
    }
    s->P.cellcap = need;
    destroy_graphs(s);
    return DB_OK;
}

db_status check_errors(db_system* s) {
    HIPCHK(s, hipGetLastError());
    // the error words come back through a pinned buffer, behind the work on
    // the stream: one synchronisation per call
    HIPCHK(s, hipMemcpyAsync(s->err_h, s->D.err, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    flush_timing(s);
    uint32_t err[4];
    std::memcpy(err, s->err_h, sizeof err);
    if (err[0] & kErrOverflow) { s->invalid = true; return fail(s, DB_EOVERFLOW, "cell capacity %u exceeded", s->P.cellcap); }
    if (err[0] & kErrFene) { s->invalid = true; return fail(s, DB_EBOND, "bond %u-%u outside its range (FENE r >= R0, tether r outside (l_min, l_max))", err[1], err[2]); }
    if (err[0] & kErrForce) { s->invalid = true; return fail(s, DB_EBOND, "force out of the representable range"); }
    if (err[0] & kErrNlist) { s->invalid = true; return fail(s, DB_EOVERFLOW, "more than %u neighbours of one particle", s->P.nlmax); }
    return DB_OK;
}

// Sweep at the current positions: buffers xcur / cell list lst, step key in slot sp.
void launch_sweep(db_system* s, int xcur, int sp) {
    const Params& P = s->P;
    const unsigned g = grid_of(P.n);
    for (int slot = 0; slot < (int)P.nrx; ++slot) {
        const unsigned gp = grid_of(P.n);       // 256 sites per workgroup
        switch (P.tpp) {
            case 1: LAUNCH(s, k_propose<1>, gp, kBlock, P, s->D, slot, xcur, sp); break;
            case 2: LAUNCH(s, k_propose<2>, gp, kBlock, P, s->D, slot, xcur, sp); break;
            case 4: LAUNCH(s, k_propose<4>, gp, kBlock, P, s->D, slot, xcur, sp); break;
            case 8: LAUNCH(s, k_propose<8>, gp, kBlock, P, s->D, slot, xcur, sp); break;
            case 16: LAUNCH(s, k_propose<16>, gp, kBlock, P, s->D, slot, xcur, sp); break;
            default: LAUNCH(s, k_propose<32>, gp, kBlock, P, s->D, slot, xcur, sp); break;
        }
        LAUNCH_EXT(s, "k_claim", k_claim, g, kBlock, P, s->D, slot, 1, xcur, sp);
        const int R = (int)s->match_rounds;
        for (int q = 2; q <= R; ++q) {
            LAUNCH(s, k_kill, g, kBlock, P, s->D, q, 0);
            LAUNCH_EXT(s, "k_claim", k_claim, g, kBlock, P, s->D, slot, q, xcur, sp);
        }
        LAUNCH(s, k_kill, g, kBlock, P, s->D, R + 1, 1);
        LAUNCH_EXT(s, "k_finish", k_finish, 1, 1024, P, s->D, slot, (R + 1) % 3, xcur, sp, s->finish_lds);
        LAUNCH_EXT(s, "k_break", k_break, g, kBlock, P, s->D, slot, xcur, sp, slot == (int)P.nrx - 1 ? 1 : 0);
    }
}

// Renumber particles in cell order (counting sort over the current cell list),
// then rebuild that cell list with the new numbers.
void launch_sort(db_system* s) {
    const Params& P = s->P;
    const unsigned gc = grid_of(P.ncell), gb = grid_of(P.ncell * P.ntypes), g = grid_of(P.n);
    const int xc = s->cur_x, f3 = (int)(s->step % 3);
    LAUNCH(s, k_clear_counts, std::min(gc, 65535u), kBlock, P, s->D, kSortList);
    LAUNCH(s, k_bin, g, kBlock, P, s->D, xc, kSortList);
    LAUNCH(s, k_cell_scan_blocks, gb, kBlock, P, s->D, kSortList);
    LAUNCH(s, k_scan_bsum, 1, 1024, s->D.cbsum, gb);
    LAUNCH(s, k_sort_assign, gb, kBlock, P, s->D, kSortList);
    LAUNCH(s, k_sort_scatter, g, kBlock, P, s->D, xc);
    LAUNCH(s, k_sort_copyback, g, kBlock, P, s->D, xc, f3);
    LAUNCH(s, k_binr, g, kBlock, P, s->D, xc, f3);
    LAUNCH(s, k_nlist, ntiles(P), kTileThreads, P, s->D, f3);
    s->tags_dirty = true;
}

// One time step t -> t+1 (plus the sweep when (t+1) % period == 0).
void launch_step(db_system* s) {
    const Params& P = s->P;
    const uint64_t t = s->step;
    const int xin = s->cur_x;
    const int sp = (int)(t & 1);
    const bool sweep = P.nrx > 0 && ((t + 1) % P.period == 0);
    const int ake = (sweep && P.kt_kinetic) ? 1 : 0;
    const unsigned gs = (unsigned)(((uint64_t)P.n * P.tpp_step + kBlock - 1) / kBlock);
    const int f3 = (int)(t % 3);
#define STEP_AS(...) LAUNCH_AS(s, "k_step", (__VA_ARGS__), gs, kBlock, P, s->D, xin, sp, f3, ake)
    if (P.ext) {
        switch (P.tpp_step) {
            case 1: STEP_AS(k_step1<true>); break;
            case 2: STEP_AS(k_step<2, 0, true>); break;
            case 4:
                if (P.qb_step == 2) STEP_AS(k_step<4, 2, true>);
                else if (P.qb_step == 4) STEP_AS(k_step<4, 4, true>);
                else STEP_AS(k_step<4, 0, true>);
                break;
            case 8: STEP_AS(k_step<8, 0, true>); break;
            case 16: STEP_AS(k_step<16, 0, true>); break;
            default: STEP_AS(k_step<32, 0, true>); break;
        }
    } else {
        switch (P.tpp_step) {
            case 1: STEP_AS(k_step1<false>); break;
            case 2: STEP_AS(k_step<2, 0, false>); break;
            case 4:
                if (P.qb_step == 2) STEP_AS(k_step<4, 2, false>);
                else if (P.qb_step == 4) STEP_AS(k_step<4, 4, false>);
                else STEP_AS(k_step<4, 0, false>);
                break;
            case 8: STEP_AS(k_step<8, 0, false>); break;
            case 16: STEP_AS(k_step<16, 0, false>); break;
            default: STEP_AS(k_step<32, 0, false>); break;
        }
    }
#undef STEP_AS
    LAUNCH(s, k_binr, grid_of(P.n), kBlock, P, s->D, xin ^ 1, (int)((t + 1) % 3));
    LAUNCH(s, k_nlist, ntiles(P), kTileThreads, P, s->D, (int)((t + 1) % 3));
    s->cur_x ^= 1;
    s->cur_list = (s->cur_list + 1) % 3;
    s->step = t + 1;
    if (sweep) launch_sweep(s, s->cur_x, (int)((t + 1) & 1));
}

// Captured graphs.  The buffer indices of a step are functions of the step
// counter t (position buffer t mod 2, cell list t mod 3, step slot t mod 2,
// rebuild-flag slot t mod 3; upload_state and every launcher keep
// cur_x = t mod 2 and cur_list = t mod 3), and whether a step ends in a
// sweep is a function of t mod period, so a graph of k steps captured at
// step t replays correctly at any step with the same t mod 6 and t mod
// period.  Kinds, so that any call replays at most a head, whole periods or
// spans, and a tail:
//   head   from an unaligned t to the next multiple of the period;
//   period one sweep period from an aligned step;
//   span   whole periods, at least 120 steps, from an aligned step;
//   tail   1 .. period - 1 steps from an aligned step;
//   step   one step (calls shorter than the head they start in);
//   sort   the spatial renumbering.
// Every graph but the spans is captured on the first db_step call (a few
// hundred steps' worth of launches), so that later calls, however short,
// replay graphs only; graphs that inter-graph gaps would otherwise multiply
// (each replay costs a few microseconds on the GPU) stay few per call.
enum : int { kGStep = 0, kGPeriod = 1, kGSpan = 2, kGSort = 3, kGHead = 4, kGTail = 5 };

bool sweep_after(const db_system* s, uint64_t t) { return s->P.nrx > 0 && (t + 1) % s->period == 0; }

// Steps in a span graph: a whole number of sweep periods, at least 120 (0:
// none, when the period alone is longer than that).
uint64_t graph_span(const db_system* s) {
    if (s->period > 120) return 0;
    return (uint64_t)s->period * ((120 + s->period - 1) / s->period);
}

// Steps in a period graph (0: none, for periods longer than 120 steps; then
// heads and tails are not used either).
uint64_t graph_period(const db_system* s) { return s->period <= 120 ? s->period : 0; }

// Steps the graph of `kind` at step t covers (len: the tail's length).
uint64_t graph_steps(const db_system* s, int kind, uint64_t t, uint64_t len) {
    switch (kind) {
        case kGStep: return 1;
        case kGPeriod: return graph_period(s);
        case kGSpan: return graph_span(s);
        case kGHead: return s->period - t % s->period;
        case kGTail: return len;
        default: return 0;
    }
}

uint64_t graph_key(const db_system* s, int kind, uint64_t t, uint64_t len) {
    uint64_t extra = 0;
    if (kind == kGStep) extra = sweep_after(s, t) ? 1 : 0;
    else if (kind == kGHead) extra = t % s->period;
    else if (kind == kGTail) extra = len;
    return ((uint64_t)kind << 48) | ((t % 6) << 32) | extra;
}

// The graph of `kind` at step t, captured (with the host's step state set to
// t and restored afterwards) when not yet held.
db_status graph_at(db_system* s, int kind, uint64_t t, uint64_t len, hipGraphExec_t* out) {
    const uint64_t key = graph_key(s, kind, t, len);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) {
        *out = it->second;
        return DB_OK;
    }
    const uint64_t step0 = s->step;
    const int x0 = s->cur_x, l0 = s->cur_list;
    const bool dirty0 = s->tags_dirty;
    s->step = t;
    s->cur_x = (int)(t & 1u);
    s->cur_list = (int)(t % 3);
    hipGraph_t g;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    if (kind == kGSort) {
        launch_sort(s);
    } else {
        const uint64_t k = graph_steps(s, kind, t, len);
        for (uint64_t q = 0; q < k; ++q) launch_step(s);
    }
    HIPCHK(s, hipStreamEndCapture(s->stream, &g));
    hipGraphExec_t ge;
    HIPCHK(s, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    HIPCHK(s, hipGraphDestroy(g));
    HIPCHK(s, hipGraphUpload(ge, s->stream));
    s->step = step0;
    s->cur_x = x0;
    s->cur_list = l0;
    s->tags_dirty = dirty0;
    s->graphs.emplace(key, ge);
    *out = ge;
    return DB_OK;
}

// Capture every graph but the spans: lcm(6, period) consecutive steps meet
// every phase a one-step or head graph can start in, and their aligned steps
// every phase of the period, tail and renumbering graphs.
db_status prepare_graphs(db_system* s) {
    const uint64_t per = s->period, t0 = s->step;
    const uint64_t l6 = 6 / std::gcd<uint64_t>(6, per) * per;
    hipGraphExec_t ge;
    db_status st;
    for (uint64_t t = t0; t < t0 + l6; ++t) {
        if ((st = graph_at(s, kGStep, t, 0, &ge)) != DB_OK) return st;
        if (!graph_period(s)) continue;
        if (t % per != 0) {
            if ((st = graph_at(s, kGHead, t, 0, &ge)) != DB_OK) return st;
            continue;
        }
        if ((st = graph_at(s, kGPeriod, t, 0, &ge)) != DB_OK) return st;
        if (s->sort_enabled && (st = graph_at(s, kGSort, t, 0, &ge)) != DB_OK) return st;
        for (uint64_t len = 1; len < per; ++len)
            if ((st = graph_at(s, kGTail, t, len, &ge)) != DB_OK) return st;
    }
    if (!graph_period(s) && s->sort_enabled)
        for (uint64_t t = t0; t < t0 + l6; ++t)
            if (t % per == 0 && (st = graph_at(s, kGSort, t, 0, &ge)) != DB_OK) return st;
    return DB_OK;
}

db_status run_batch(db_system* const* systems, uint32_t count, uint64_t nsteps, const db_batch_plan& plan,
                    float* ms);

// Small systems advanced by many steps in one call can run as a batch of one
// (one 1024-thread workgroup runs every step, barriers in place of kernel
// launches; bitwise the same trajectory).  Which is faster depends on the
// system, not only on its size: a 512-particle dimer gas at density 0.1
// takes 9.5 us per step that way against 12.5 us on the grid kernels, but
// sweep replicas of 257 to 684 particles at densities 0.08 to 0.39 take
// 12.8 to 18.8 us against 12.0 to 14.3 us.  So the first call of at least
// 2 kPathTrial steps on such a system runs kPathTrial steps on each path
// between events, and the end of that call keeps the faster path for every
// later call (path_pick).  kPathTrial stays below the shortest span graph
// (120 steps), so the grid's part replays only graphs captured before the
// first event (prepare_graphs; spans are captured when first used, and a
// capture inside the timed part would leave the GPU idle and count against
// the grid).  Above kOneGroupMaxN particles one CU is slower than
// the whole GPU (sweep replicas of 800 to 1030 particles: 15.6 to 19.3 us
// against 12.4 to 14.5); below kOneGroupMinSteps steps per call the batch's
// per-call set-up is not repaid.  Neither path is measured or taken with a
// caller-chosen launch shape, with graphs off or with kernel timing on.
constexpr uint32_t kOneGroupMaxN = 768;
constexpr uint64_t kOneGroupMinSteps = 200;
constexpr uint64_t kPathTrial = 100;
static_assert(kPathTrial < 120, "the grid's timed part must not need a span graph");

db_status run_one_group(db_system* s, uint64_t nsteps) {
    db_batch_plan plan{};
    plan.n_classes = 1;
    plan.n_max[0] = 0xFFFFFFFFu;
    plan.threads[0] = (uint32_t)kBatchMaxThreads;
    db_system* one[1] = {s};
    return run_batch(one, 1, nsteps, plan, nullptr);
}

db_status run_grid(db_system* s, uint64_t nsteps);

db_status run_steps(db_system* s, uint64_t nsteps) {
    const bool small = s->use_graphs && !s->timing.on && s->tpp_user == 0 && s->n <= kOneGroupMaxN &&
                       nsteps >= kOneGroupMinSteps;
    if (!small || s->path_pick == 2) return run_grid(s, nsteps);
    if (s->path_pick == 0 && !s->path_pending && nsteps >= 2 * kPathTrial) {
        // the grid's graphs are captured before the first event, so that
        // their set-up is not timed
        for (auto& e : s->path_ev)
            if (!e) HIPCHK(s, hipEventCreate(&e));
        if (s->graphs.empty()) {
            const db_status st = prepare_graphs(s);
            if (st != DB_OK) return st;
        }
        HIPCHK(s, hipEventRecord(s->path_ev[0], s->stream));
        db_status st = run_grid(s, kPathTrial);
        if (st != DB_OK) return st;
        HIPCHK(s, hipEventRecord(s->path_ev[1], s->stream));
        st = run_one_group(s, kPathTrial);
        if (st != DB_OK) return st;
        HIPCHK(s, hipEventRecord(s->path_ev[2], s->stream));
        s->path_pending = true;
        nsteps -= 2 * kPathTrial;
    }
    if (nsteps == 0) return DB_OK;
    return nsteps >= kOneGroupMinSteps ? run_one_group(s, nsteps) : run_grid(s, nsteps);
}

// After a call that measured both paths has synchronised: keep the faster.
void settle_path(db_system* s) {
    if (!s->path_pending) return;
    s->path_pending = false;
    float grid_ms = 0.f, one_ms = 0.f;
    if (hipEventElapsedTime(&grid_ms, s->path_ev[0], s->path_ev[1]) != hipSuccess ||
        hipEventElapsedTime(&one_ms, s->path_ev[1], s->path_ev[2]) != hipSuccess) {
        (void)hipGetLastError();           // measured again by a later call
        return;
    }
    s->path_pick = one_ms <= grid_ms ? 1 : 2;
}

db_status run_grid(db_system* s, uint64_t nsteps) {
    const uint64_t span = graph_span(s), per = graph_period(s);
    const bool graphs = s->use_graphs && !s->timing.on;
    if (graphs && s->graphs.empty()) {
        const db_status st = prepare_graphs(s);
        if (st != DB_OK) return st;
    }
    uint64_t done = 0;
    while (done < nsteps) {
        const bool aligned = (s->step % s->period) == 0;
        // renumbering at the first sweep-period boundary once it is due
        if (aligned && s->sort_enabled && s->step >= s->sort_due) {
            if (graphs) {
                hipGraphExec_t ge;
                const db_status st = graph_at(s, kGSort, s->step, 0, &ge);
                if (st != DB_OK) return st;
                HIPCHK(s, hipGraphLaunch(ge, s->stream));
            } else {
                launch_sort(s);
            }
            s->tags_dirty = true;
            s->sort_due = s->step + kSortPeriod;
        }
        if (!graphs) {
            launch_step(s);
            ++done;
            continue;
        }
        const uint64_t left = nsteps - done;
        int kind = kGStep;
        uint64_t len = 0;
        if (per && !aligned) {
            if (left >= per - s->step % per) kind = kGHead;
        } else if (aligned && span && left >= span) {
            kind = kGSpan;
        } else if (aligned && per && left >= per) {
            kind = kGPeriod;
        } else if (aligned && per) {
            kind = kGTail;
            len = left;
        }
        const uint64_t k = graph_steps(s, kind, s->step, len);
        hipGraphExec_t ge;
        const db_status st = graph_at(s, kind, s->step, len, &ge);
        if (st != DB_OK) return st;
        HIPCHK(s, hipGraphLaunch(ge, s->stream));
        s->step += k;
        s->cur_x = (int)(s->step & 1u);
        s->cur_list = (int)(s->step % 3);
        done += k;
    }
    return DB_OK;
}

db_status ready(db_system* s) {
    if (!s) return DB_EINVAL;
    if (s->dead) return fail(s, DB_EDEVICE, "device error earlier on this handle");
    if (!s->committed) return fail(s, DB_ESTATE, "system not committed");
    if (s->invalid) return fail(s, DB_ESTATE, "state invalid after an error; call db_set_state");
    return DB_OK;
}

// Checks shared by db_set_state and db_load_checkpoint: positions inside the
// box, and dynamic bonds that a reaction of the system could have made
// (matching types, distinct tags, valences held, each pair once).
db_status check_state(db_system* s, const float* pos3, const uint32_t* pairs, const uint32_t* bts,
                             uint64_t m) {
    const float half = (float)(0.5 * s->L);
    for (size_t k = 0; k < 3 * (size_t)s->n; ++k)
        if (!(pos3[k] >= -half && pos3[k] < half)) return fail(s, DB_EINVAL, "position %zu outside [-L/2, L/2)", k / 3);
    std::vector<int> bt2rx(s->bonds.size(), -1);
    for (size_t a = 0; a < s->rx.size(); ++a) bt2rx[s->rx[a].bond_type] = (int)a;
    std::vector<uint32_t> occ(s->n, 0);
    std::vector<uint64_t> keys;
    keys.reserve(m);
    for (uint64_t k = 0; k < m; ++k) {
        uint32_t a = pairs[2 * k], b = pairs[2 * k + 1];
        if (a >= s->n || b >= s->n || a == b) return fail(s, DB_EINVAL, "dynamic bond %llu: bad tags", (unsigned long long)k);
        if (bts[k] >= bt2rx.size() || bt2rx[bts[k]] < 0)
            return fail(s, DB_EINVAL, "dynamic bond %llu: bond type is not a reaction's", (unsigned long long)k);
        const auto& d = s->rx[bt2rx[bts[k]]];
        const uint32_t ta = s->type[a], tb = s->type[b];
        if (!((ta == d.type_a && tb == d.type_b) || (ta == d.type_b && tb == d.type_a)))
            return fail(s, DB_EINVAL, "dynamic bond %llu: types do not match its reaction", (unsigned long long)k);
        if (++occ[a] > s->types[ta].valence || ++occ[b] > s->types[tb].valence)
            return fail(s, DB_EINVAL, "dynamic bond %llu exceeds a valence", (unsigned long long)k);
        keys.push_back(((uint64_t)std::min(a, b) << 32) | std::max(a, b));
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return fail(s, DB_EINVAL, "duplicate dynamic bond");
    return DB_OK;
}

// ---------------------------------------------------------------- checkpoints
// Layout (little-endian): a 48-byte header {magic, version, n, reactions,
// step, dynamic bonds m, configuration fingerprint, payload hash}, then the
// payload: cumulative counters (3 x reactions uint64: attempts, forms,
// breaks), positions (3n float, tag order), the integrator's carried
// velocities u (3n float), periodic image counters (3n int32), the bond pairs
// (2m uint32, tag_lo < tag_hi) and their bond types (m uint32).
constexpr uint32_t kCkptMagic = 0x4B434244u;   // "DBCK"
constexpr uint32_t kCkptVersion = 1u;
constexpr uint64_t kCkptHeader = 48;

struct Fnv {
    uint64_t h = 0xcbf29ce484222325ull;
    void bytes(const void* p, size_t k) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < k; ++i) { h ^= c[i]; h *= 0x100000001b3ull; }
    }
    template <class T> void val(T v) { bytes(&v, sizeof v); }
};

// Everything set up before db_commit (and the integrator settings) that the
// trajectory depends on; launch shapes, the list skin, cell capacity, the
// matching schedule and renumbering do not change results and are left out.
uint64_t config_fingerprint(const db_system* s) {
    Fnv f;
    f.val(s->n); f.val(s->ntypes); f.val(s->L); f.val(s->seed);
    for (const auto& t : s->types) { f.val(t.valence); f.val(t.sigma); f.val(t.eps); f.val(t.mass); }
    for (const auto& b : s->bonds) {
        f.val((int32_t)b.kind); f.val(b.k); f.val(b.r0); f.val(b.lmin); f.val(b.lc1); f.val(b.lc0); f.val(b.lmax);
    }
    for (const auto& r : s->rx) {
        f.val(r.type_a); f.val(r.type_b); f.val(r.bond_type); f.val(r.r_min); f.val(r.r_max);
        f.val(r.k_on); f.val(r.k_off); f.val(r.epsilon); f.val(r.p_on0); f.val(r.self_avoid);
    }
    for (const auto& md : s->mods) { f.val((int32_t)md.kind); f.val(md.lam); f.val(md.tm); f.val(md.k_on_m); f.val(md.k_off_m); f.val(md.a); }
    f.bytes(s->type.data(), s->type.size() * 4);
    f.bytes(s->stat_pairs.data(), s->stat_pairs.size() * 4);
    f.bytes(s->stat_bt.data(), s->stat_bt.size() * 4);
    f.val(s->dt); f.val(s->kT); f.val(s->gamma); f.val(s->period); f.val((int32_t)s->kt_source);
    return f.h;
}

uint64_t ckpt_size(uint32_t n, uint32_t nrx, uint64_t m) {
    return kCkptHeader + 24ull * nrx + 36ull * n + 12ull * m;
}

db_status sync_tags(db_system* s) {
    if (!s->tags_dirty) return DB_OK;
    HIPCHK(s, hipMemcpyAsync(s->tag_h.data(), s->D.tag, s->n * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->rtag_h.data(), s->D.rtag, s->n * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->tags_dirty = false;
    return DB_OK;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

db_status db_create(uint32_t n, uint32_t n_types, double box_L, uint32_t seed, int device, db_system** out) {
    if (!out) return fail(nullptr, DB_EINVAL, "out is NULL");
    *out = nullptr;
    if (n == 0 || n >= (1u << 24)) return fail(nullptr, DB_EINVAL, "n must be in [1, 2^24)");
    if (n_types == 0 || n_types > (uint32_t)kMaxTypes) return fail(nullptr, DB_EINVAL, "n_types must be in [1, 8]");
    if (!(box_L > 0.0) || !std::isfinite(box_L)) return fail(nullptr, DB_EINVAL, "box_L must be positive");
    db_system* s = new (std::nothrow) db_system();
    if (!s) return fail(nullptr, DB_ENOMEM, "out of host memory");
    s->n = n;
    s->ntypes = n_types;
    s->L = box_L;
    s->seed = seed;
    s->device = device;
    s->types.assign(n_types, TypeCfg{});
    s->tag_h.resize(n);
    s->rtag_h.resize(n);
    std::iota(s->tag_h.begin(), s->tag_h.end(), 0u);
    std::iota(s->rtag_h.begin(), s->rtag_h.end(), 0u);
    *out = s;
    return DB_OK;
}

void db_destroy(db_system* s) {
    if (!s) return;
    if (s->committed) {
        (void)hipSetDevice(s->device);
        (void)hipStreamSynchronize(s->stream);
        destroy_graphs(s);
        for (auto& p : s->timing.pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto e : s->timing.pool) (void)hipEventDestroy(e);
        if (s->ev_out) (void)hipEventDestroy(s->ev_out);
        if (s->ev_back) (void)hipEventDestroy(s->ev_back);
        for (auto e : s->path_ev)
            if (e) (void)hipEventDestroy(e);
        if (s->err_h) (void)hipHostFree(s->err_h);
        for (void* p : s->allocs) (void)hipFree(p);
        if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    }
    delete s;
}

db_status db_set_type(db_system* s, uint32_t type, uint32_t valence, double sigma, double eps, double mass) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "parameters are fixed after commit");
    if (type >= s->ntypes) return fail(s, DB_EINVAL, "type out of range");
    if (valence > (uint32_t)kMaxValence) return fail(s, DB_EINVAL, "valence above %d", kMaxValence);
    if (!(sigma >= 0.0) || !(eps >= 0.0) || !(mass > 0.0) || !std::isfinite(sigma) || !std::isfinite(mass))
        return fail(s, DB_EINVAL, "sigma, eps must be >= 0 and mass > 0");
    s->types[type] = TypeCfg{valence, sigma, eps, mass};
    s->validated = false;
    return DB_OK;
}

db_status db_set_particles(db_system* s, const float* pos3, const float* vel3, const uint32_t* type) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "use db_set_state after commit");
    if (!pos3 || !type) return fail(s, DB_EINVAL, "pos3 and type are required");
    const float half = (float)(0.5 * s->L);
    for (size_t k = 0; k < 3 * (size_t)s->n; ++k)
        if (!(pos3[k] >= -half && pos3[k] < half)) return fail(s, DB_EINVAL, "position %zu outside [-L/2, L/2)", k / 3);
    for (uint32_t i = 0; i < s->n; ++i)
        if (type[i] >= s->ntypes) return fail(s, DB_EINVAL, "type of particle %u out of range", i);
    s->pos.assign(pos3, pos3 + 3 * (size_t)s->n);
    if (vel3) s->vel.assign(vel3, vel3 + 3 * (size_t)s->n);
    else s->vel.clear();
    s->vel_given = vel3 != nullptr;
    s->type.assign(type, type + s->n);
    s->have_particles = true;
    s->validated = false;
    return DB_OK;
}

db_status db_add_bond_type(db_system* s, db_bond_kind kind, double k, double r0, uint32_t* id) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "parameters are fixed after commit");
    if (kind != DB_BOND_HARMONIC && kind != DB_BOND_FENE) return fail(s, DB_EINVAL, "unknown bond kind");
    if (s->bonds.size() >= (size_t)kMaxBondTypes) return fail(s, DB_EINVAL, "too many bond types");
    if (!(k >= 0.0) || !(r0 >= 0.0) || !std::isfinite(k) || !std::isfinite(r0) || (kind == DB_BOND_FENE && !(r0 > 0.0)))
        return fail(s, DB_EINVAL, "bond parameters out of range");
    s->bonds.push_back(BondCfg{kind, k, r0});
    if (id) *id = (uint32_t)s->bonds.size() - 1;
    s->validated = false;
    return DB_OK;
}

db_status db_add_tether_bond_type(db_system* s, double k_b, double l_min, double l_c1, double l_c0, double l_max,
                                  uint32_t* id) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "parameters are fixed after commit");
    if (s->bonds.size() >= (size_t)kMaxBondTypes) return fail(s, DB_EINVAL, "too many bond types");
    for (double v : {k_b, l_min, l_c1, l_c0, l_max})
        if (!std::isfinite(v)) return fail(s, DB_EINVAL, "tether parameters must be finite");
    if (!(k_b >= 0.0) || !(l_min >= 0.0) || !(l_min < l_c1) || !(l_c1 < l_c0) || !(l_c0 < l_max))
        return fail(s, DB_EINVAL, "tether needs k_b >= 0 and 0 <= l_min < l_c1 < l_c0 < l_max");
    BondCfg b{DB_BOND_TETHER, k_b, 0.5 * (l_c1 + l_c0)};
    b.lmin = l_min;
    b.lc1 = l_c1;
    b.lc0 = l_c0;
    b.lmax = l_max;
    s->bonds.push_back(b);
    if (id) *id = (uint32_t)s->bonds.size() - 1;
    s->validated = false;
    return DB_OK;
}

db_status db_set_reaction_melting(db_system* s, uint32_t reaction, double lambda, double T_melt, double k_on_melt,
                                  double k_off_melt) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "reactions are fixed after commit");
    if (reaction >= s->rx.size()) return fail(s, DB_EINVAL, "no reaction %u", reaction);
    if (s->mods[reaction].kind == 2) return fail(s, DB_EINVAL, "melting and slip modifiers are mutually exclusive");
    if (!(lambda >= 0.0) || !std::isfinite(lambda) || !std::isfinite(T_melt) || !(k_on_melt >= 0.0) ||
        !(k_off_melt >= 0.0) || !std::isfinite(k_on_melt) || !std::isfinite(k_off_melt))
        return fail(s, DB_EINVAL, "melting needs lambda >= 0, finite T_melt, melted rates >= 0");
    RxMod& m = s->mods[reaction];
    m = RxMod{};
    m.kind = 1;
    m.lam = lambda;
    m.tm = T_melt;
    m.k_on_m = k_on_melt;
    m.k_off_m = k_off_melt;
    s->validated = false;
    return DB_OK;
}

db_status db_set_reaction_slip(db_system* s, uint32_t reaction, double a) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "reactions are fixed after commit");
    if (reaction >= s->rx.size()) return fail(s, DB_EINVAL, "no reaction %u", reaction);
    if (s->mods[reaction].kind == 1) return fail(s, DB_EINVAL, "melting and slip modifiers are mutually exclusive");
    if (!(a >= 0.0) || !std::isfinite(a)) return fail(s, DB_EINVAL, "slip coefficient must be finite and >= 0");
    RxMod& m = s->mods[reaction];
    m = RxMod{};
    m.kind = 2;
    m.a = a;
    s->validated = false;
    return DB_OK;
}

db_status db_add_static_bonds(db_system* s, const uint32_t* pairs, const uint32_t* bt, uint64_t m) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "static bonds are fixed after commit");
    if (m && (!pairs || !bt)) return fail(s, DB_EINVAL, "NULL arrays");
    s->stat_pairs.insert(s->stat_pairs.end(), pairs, pairs + 2 * m);
    s->stat_bt.insert(s->stat_bt.end(), bt, bt + m);
    s->validated = false;
    return DB_OK;
}

db_status db_add_reaction(db_system* s, const db_reaction_desc* d, uint32_t* id) {
    if (!s || !d) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "reactions are fixed after commit");
    if (s->rx.size() >= (size_t)kMaxRx) return fail(s, DB_EINVAL, "at most %d reactions", kMaxRx);
    s->rx.push_back(*d);
    s->mods.push_back(RxMod{});
    if (id) *id = (uint32_t)s->rx.size() - 1;
    s->validated = false;
    return DB_OK;
}

db_status db_set_integrator(db_system* s, double dt, double kT, double gamma, uint32_t period, db_kt_source kt_source) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "integrator is fixed after commit");
    if (!(dt > 0.0) || !(kT >= 0.0) || !(gamma >= 0.0) || period < 1 || !std::isfinite(dt) ||
        !std::isfinite(kT) || !std::isfinite(gamma))
        return fail(s, DB_EINVAL, "dt > 0, kT >= 0, gamma >= 0, period >= 1 required");
    if (kt_source != DB_KT_SETPOINT && kt_source != DB_KT_KINETIC) return fail(s, DB_EINVAL, "bad kt_source");
    s->dt = dt;
    s->kT = kT;
    s->gamma = gamma;
    s->period = period;
    s->kt_source = kt_source;
    s->validated = false;
    return DB_OK;
}

db_status db_set_temperature(db_system* s, double kT) {
    if (!s) return DB_EINVAL;
    if (!(kT >= 0.0) || !std::isfinite(kT)) return fail(s, DB_EINVAL, "kT must be finite and >= 0");
    if (!s->committed) {
        s->kT = kT;
        s->validated = false;
        return DB_OK;
    }
    if (s->dead) return fail(s, DB_EDEVICE, "device error earlier on this handle");
    HIPCHK(s, hipSetDevice(s->device));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->kT = kT;
    apply_temperature(s);
    StepTabs th;
    fill_tabs(s, th);
    HIPCHK(s, hipMemcpy((void*)s->D.tabs, &th, sizeof th, hipMemcpyHostToDevice));
    destroy_graphs(s);
    return DB_OK;
}

db_status db_set_cell_capacity(db_system* s, uint32_t slots) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "cell capacity is fixed after commit");
    if (slots > 1024) return fail(s, DB_EINVAL, "cell capacity above 1024");
    s->cellcap_user = slots;
    return DB_OK;
}

db_status db_set_neighbor_list(db_system* s, double skin, uint32_t max_neighbors) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "neighbour list is fixed after commit");
    if (!std::isfinite(skin) || skin > 100.0) return fail(s, DB_EINVAL, "skin out of range");
    if (max_neighbors > 1024) return fail(s, DB_EINVAL, "max_neighbors above 1024");
    s->skin = skin < 0.0 ? kDefaultSkin : skin;
    s->nlmax_user = max_neighbors;
    return DB_OK;
}

db_status db_set_matching(db_system* s, uint32_t grid_rounds, uint32_t lds_limit) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "matching schedule is fixed after commit");
    if (grid_rounds < 1 || grid_rounds > 8) return fail(s, DB_EINVAL, "grid_rounds must be in [1, 8]");
    if (lds_limit > kFinishLds) return fail(s, DB_EINVAL, "lds_limit above %u", kFinishLds);
    s->match_rounds = grid_rounds;
    s->finish_lds = lds_limit;
    return DB_OK;
}

db_status db_set_step_shape(db_system* s, uint32_t tpp, uint32_t list_batch) {
    if (!s) return DB_EINVAL;
    if (tpp != 0 && tpp != 1 && tpp != 2 && tpp != 4 && tpp != 8 && tpp != 16 && tpp != 32)
        return fail(s, DB_EINVAL, "threads per particle must be 0 (automatic), 1, 2, 4, 8, 16 or 32");
    if (list_batch != 0 && list_batch != 1 && list_batch != 2 && list_batch != 4)
        return fail(s, DB_EINVAL, "list batch must be 0 (automatic), 1, 2 or 4");
    if (s->dead) return fail(s, DB_EDEVICE, "device error earlier on this handle");
    s->tpp_user = tpp;
    s->qb_user = list_batch;
    if (s->committed) {
        HIPCHK(s, hipSetDevice(s->device));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        destroy_graphs(s);
        s->P.tpp_step = tpp ? tpp : auto_step_tpp(s->n);
        s->P.tpp = tpp ? tpp : auto_propose_tpp(s->n);
        s->P.qb_step = s->P.tpp_step == 4 ? list_batch : 0u;
    }
    return DB_OK;
}

db_status db_get_step_shape(const db_system* s, uint32_t* tpp, uint32_t* list_batch) {
    if (!s || !tpp || !list_batch) return DB_EINVAL;
    *tpp = s->committed ? s->P.tpp_step : s->tpp_user;
    *list_batch = s->committed ? (s->P.qb_step ? s->P.qb_step : (s->P.tpp_step == 1 ? 4u : std::max(1u, 4u / s->P.tpp_step)))
                               : s->qb_user;
    return DB_OK;
}

db_status db_validate(db_system* s) {
    if (!s) return DB_EINVAL;
    return validate(s);
}

db_status db_get_reaction(const db_system* s, uint32_t id, db_reaction_desc* out, double* p_on0, double* p_off0) {
    if (!s || !out) return DB_EINVAL;
    if (!s->validated) return DB_ESTATE;
    if (id >= s->rx.size()) return DB_EINVAL;
    *out = s->rx[id];
    out->k_on = s->res[id].k_on;
    out->k_off = s->res[id].k_off;
    out->epsilon = s->res[id].eps;
    out->p_on0 = s->res[id].p_on;
    if (p_on0) *p_on0 = s->res[id].p_on;
    if (p_off0) *p_off0 = s->res[id].p_off;
    return DB_OK;
}

static db_status commit_impl(db_system* s);

db_status db_commit(db_system* s) {
    if (!s) return DB_EINVAL;
    if (s->committed) return fail(s, DB_ESTATE, "already committed");
    const db_status st = commit_impl(s);
    if (st != DB_OK && s->committed && st != DB_EBOND && st != DB_EOVERFLOW) s->dead = true;
    return st;
}

static db_status commit_impl(db_system* s) {
    if (s->committed) return fail(s, DB_ESTATE, "already committed");
    db_status st = validate(s);
    if (st != DB_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(s, DB_EDEVICE, "no HIP device available");
    }
    if (s->device < 0 || s->device >= ndev) return fail(s, DB_EDEVICE, "device %d not present", s->device);
    HIPCHK(s, hipSetDevice(s->device));
    fill_params(s);
    const uint32_t n = s->n;
    // a sweep forms at most one bond per site and reaction (n / 2 per
    // reaction) and breaks only bonds present at its start (at most
    // cap_max n / 2)
    s->P.evcap[0] = std::max(s->P.nrx * (n / 2), 1u);
    s->P.evcap[1] = std::max((uint32_t)(((uint64_t)s->P.cap_max * n) / 2), 1u);
    const Params& P = s->P;
    Dev& D = s->D;
    HIPCHK(s, hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
    s->stream = s->own_stream;
    s->committed = true;   // from here on db_destroy frees device memory
    {
        PairTab* pt = nullptr;
        DALLOC(s, pt, (size_t)kMaxTypes * kMaxTypes);
        HIPCHK(s, hipMemcpyAsync(pt, s->pair_h.data(), s->pair_h.size() * sizeof(PairTab),
                                 hipMemcpyHostToDevice, s->stream));
        D.pair = pt;
        // step tables: the same numbers k_step would read from the parameter
        // block, laid out for one 16-byte copy per thread into LDS
        StepTabs th{};
        fill_tabs(s, th);
        StepTabs* tt = nullptr;
        DALLOC(s, tt, 1);
        HIPCHK(s, hipMemcpy(tt, &th, sizeof th, hipMemcpyHostToDevice));
        D.tabs = tt;
    }
    DALLOC(s, D.x[0], n);
    DALLOC(s, D.x[1], n);
    DALLOC(s, D.u, n);
    DALLOC(s, D.img, 3 * (size_t)n);
    DALLOC(s, D.tag, n);
    DALLOC(s, D.rtag, n);
    DALLOC(s, D.occ, n);
    DALLOC(s, D.dyn, (size_t)P.cap_max * n);
    DALLOC(s, D.stat, (size_t)std::max(P.stat_max, 1u) * n);
    DALLOC(s, D.mol, n);
    for (int l = 0; l < 3; ++l) {
        DALLOC(s, D.ccount[l], P.ncell);
        DALLOC(s, D.cpos[l], (size_t)P.ncell * P.cellcap);
        DALLOC(s, D.best[l], n);
    }
    DALLOC(s, D.prop, n);
    DALLOC(s, D.key, n);
    DALLOC(s, D.estate, n);
    DALLOC(s, D.claimed, n);
    DALLOC(s, D.live, n);
    DALLOC(s, D.live_count, 4);
    DALLOC(s, D.ev[0], P.evcap[0]);
    DALLOC(s, D.ev[1], P.evcap[1]);
    DALLOC(s, D.evc, 4);
    DALLOC(s, D.counters, (size_t)3 * kMaxRx * kCtrSlots);
    DALLOC(s, D.stepv, 2);
    DALLOC(s, D.ke_fix, 2);
    DALLOC(s, D.err, 4);
    DALLOC(s, D.f4, 2 * (size_t)n);
    DALLOC(s, D.red, 4 + kMaxRx);
    DALLOC(s, s->ana, kAnaWords);
    DALLOC(s, D.scan, (size_t)n + 1);
    DALLOC(s, D.parent, n);
    DALLOC(s, s->bsum, grid_of(n) + 1);
    DALLOC(s, D.nl, (size_t)P.nlmax * n);
    DALLOC(s, D.nl_cnt, n);
    DALLOC(s, D.xref, n);
    DALLOC(s, D.rflag, 8);
    HIPCHK(s, hipMemsetAsync(D.rflag, 0, 8 * sizeof(uint32_t), s->stream));
    DALLOC(s, D.corder, P.ncell);
    DALLOC(s, D.newidx, n);
    DALLOC(s, D.cstart, (size_t)P.ncell * P.ntypes + 1);
    DALLOC(s, D.cbsum, grid_of(P.ncell * P.ntypes) + 1);
    DALLOC(s, D.x_alt, n);
    DALLOC(s, D.u_alt, n);
    DALLOC(s, D.img_alt, 3 * (size_t)n);
    DALLOC(s, D.tag_alt, n);
    DALLOC(s, D.occ_alt, n);
    DALLOC(s, D.mol_alt, n);
    DALLOC(s, D.dyn_alt, (size_t)P.cap_max * n);
    DALLOC(s, D.stat_alt, (size_t)std::max(P.stat_max, 1u) * n);
    DALLOC(s, s->stage, n);
    DALLOC(s, s->flag, 1);
    {
        void* h = nullptr;
        if (hipHostMalloc(&h, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(s, DB_ENOMEM, "pinned host allocation failed");
        }
        s->err_h = (uint32_t*)h;
    }
    // static topology, molecule ids, tags
    std::vector<uint32_t> stat((size_t)std::max(P.stat_max, 1u) * n, kEmpty), fillc(n, 0);
    for (size_t k = 0; k < s->stat_bt.size(); ++k) {
        const uint32_t i = s->stat_pairs[2 * k], j = s->stat_pairs[2 * k + 1], b = s->stat_bt[k];
        stat[(size_t)fillc[i]++ * n + i] = j | (b << 24);
        stat[(size_t)fillc[j]++ * n + j] = i | (b << 24);
    }
    std::vector<uint32_t> mol;
    union_find_mol(s, mol);
    HIPCHK(s, hipMemcpyAsync(D.stat, stat.data(), stat.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(D.mol, mol.data(), n * 4, hipMemcpyHostToDevice, s->stream));
    {
        const std::vector<uint32_t> co = morton_cells(P.nc);
        HIPCHK(s, hipMemcpy(D.corder, co.data(), co.size() * 4, hipMemcpyHostToDevice));
    }
    HIPCHK(s, hipMemcpyAsync(D.tag, s->tag_h.data(), n * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(D.rtag, s->rtag_h.data(), n * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(D.counters, 0, (size_t)3 * kMaxRx * kCtrSlots * sizeof(unsigned long long), s->stream));
    for (int l = 0; l < 3; ++l) HIPCHK(s, hipMemsetAsync(D.best[l], 0xFF, (size_t)n * 8, s->stream));
    HIPCHK(s, hipMemsetAsync(D.estate, 0, n, s->stream));
    HIPCHK(s, hipMemsetAsync(D.claimed, 0, n, s->stream));
    HIPCHK(s, hipMemsetAsync(D.prop, 0xFF, (size_t)n * 4, s->stream));
    HIPCHK(s, hipMemsetAsync(D.live_count, 0, 16, s->stream));
    HIPCHK(s, hipMemsetAsync(D.newidx, 0, (size_t)n * 4, s->stream));   // in range before any sort
    HIPCHK(s, hipMemsetAsync(D.nl, 0, (size_t)P.nlmax * n * 4, s->stream));
    HIPCHK(s, hipMemsetAsync(D.nl_cnt, 0, (size_t)n * 4, s->stream));
    s->step = 0;
    return upload_state(s, s->pos.data(), s->vel.data(), nullptr, nullptr, 0);
}

db_status db_step(db_system* s, uint64_t nsteps) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    HIPCHK(s, hipSetDevice(s->device));
    st = run_steps(s, nsteps);
    if (st != DB_OK) return st;
    st = check_errors(s);
    if (st == DB_OK) settle_path(s);
    return st;
}

}  // extern "C"

namespace {

// launch plans of db_step_batch stored per device
std::mutex g_plan_mu;
std::map<int, db_batch_plan> g_plans;

db_batch_plan default_plan() {
    db_batch_plan p{};
    p.n_classes = 1;
    p.n_max[0] = 0xFFFFFFFFu;
    p.threads[0] = (uint32_t)kBatchMaxThreads;
    return p;
}

const char* plan_error(const db_batch_plan* p) {
    if (!p) return "null plan";
    if (p->n_classes < 1 || p->n_classes > DB_BATCH_MAX_CLASSES) return "plan: n_classes must be in [1, 8]";
    for (uint32_t k = 0; k < p->n_classes; ++k) {
        if (p->threads[k] < 64 || p->threads[k] > (uint32_t)kBatchMaxThreads || p->threads[k] % 64u)
            return "plan: threads must be a multiple of 64 in [64, 1024]";
        if (k && p->n_max[k] <= p->n_max[k - 1]) return "plan: n_max must ascend";
    }
    return nullptr;
}

uint32_t class_of(const db_batch_plan& p, uint32_t n) {
    for (uint32_t k = 0; k + 1 < p.n_classes; ++k)
        if (n <= p.n_max[k]) return k;
    return p.n_classes - 1;
}

bool device_ok(int device) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return device >= 0 && device < ndev;
}

db_status batch_check(db_system* const* systems, uint32_t count) {
    if (!systems || count == 0) return DB_EINVAL;
    for (uint32_t k = 0; k < count; ++k) {
        db_status st = ready(systems[k]);
        if (st != DB_OK) return st;
        for (uint32_t q = 0; q < k; ++q)
            if (systems[q] == systems[k]) return fail(systems[k], DB_EINVAL, "system listed twice in a batch");
        if (systems[k]->device != systems[0]->device)
            return fail(systems[k], DB_EINVAL, "batched systems must share one device");
    }
    return DB_OK;
}

// Device buffers, streams, events and graph of one batch run, released on
// every exit path.
struct BatchRun {
    BatchItem* items = nullptr;
    BatchState* state = nullptr;
    std::vector<hipStream_t> streams;      // extra streams of the 2nd, 3rd ... occupied class
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchRun() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t q : streams) (void)hipStreamDestroy(q);
        if (items) (void)hipFree(items);
        if (state) (void)hipFree(state);
    }
    hipEvent_t event() {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        events.push_back(e);
        return e;
    }
};

constexpr uint32_t kBatchChunk = 2000;     // steps per launch

// Every system advanced by nsteps under `plan`; *ms (may be null) receives
// the device time of the graph.  On a device error every system is marked
// dead; per-system errors are checked afterwards.
db_status run_batch(db_system* const* systems, uint32_t count, uint64_t nsteps, const db_batch_plan& plan,
                    float* ms) {
    db_system* s0 = systems[0];
    if (ms) *ms = 0.0f;
    HIPCHK(s0, hipSetDevice(s0->device));
    for (uint32_t k = 0; k < count; ++k) HIPCHK(systems[k], hipStreamSynchronize(systems[k]->stream));
    if (nsteps == 0) return DB_OK;
    // classes in plan order; largest systems first inside a class, so that
    // their workgroups start in the first wave
    // groups: (class, kernel variant); systems with tether bonds or rate
    // modifiers run the full variant of the kernel
    std::vector<std::vector<uint32_t>> groups(2 * plan.n_classes);
    for (uint32_t k = 0; k < count; ++k)
        groups[2 * class_of(plan, systems[k]->n) + (systems[k]->P.ext ? 1 : 0)].push_back(k);
    std::vector<uint32_t> order;
    std::vector<std::pair<uint32_t, uint32_t>> spans;    // (offset, size) of each occupied group
    std::vector<uint32_t> threads, full;
    for (uint32_t g = 0; g < 2 * plan.n_classes; ++g) {
        auto& v = groups[g];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) { return systems[a]->n > systems[b]->n; });
        spans.emplace_back((uint32_t)order.size(), (uint32_t)v.size());
        threads.push_back(plan.threads[g / 2]);
        full.push_back(g & 1u);
        order.insert(order.end(), v.begin(), v.end());
    }
    // Positions in LDS (the LX variant of k_batch) wherever the largest
    // system of a group fits in the LDS share its workgroup has anyway: the
    // registers of a step let one 1024-thread workgroup, two of 512 or four
    // of 256 share a CU.
    std::vector<size_t> xlds(spans.size(), 0);
    for (size_t g = 0; g < spans.size(); ++g) {
        const size_t nmax = systems[order[spans[g].first]]->n;
        const size_t share = (size_t)kBatchLdsTotal * threads[g] / kBatchMaxThreads;
        if (nmax * sizeof(float4) + kBatchLdsStatic <= share) xlds[g] = nmax * sizeof(float4);
    }
    std::vector<BatchItem> items(count);
    std::vector<BatchState> state(count);
    for (uint32_t k = 0; k < count; ++k) {
        const db_system* s = systems[order[k]];
        items[k].P = s->P;
        items[k].D = s->D;
        state[k].t = s->step;
        state[k].cur_x = s->cur_x;
        state[k].cur_list = s->cur_list;
    }
    db_status st = DB_OK;
    {
        BatchRun R;
        auto dev_fail = [&](const char* what) {
            for (uint32_t k = 0; k < count; ++k) systems[k]->dead = true;
            return fail(s0, DB_EDEVICE, "batch: %s", what);
        };
        if (hipMalloc(&R.items, count * sizeof(BatchItem)) != hipSuccess ||
            hipMalloc(&R.state, count * sizeof(BatchState)) != hipSuccess)
            return fail(s0, DB_ENOMEM, "batch: device allocation failed");
        if (hipMemcpyAsync(R.items, items.data(), count * sizeof(BatchItem), hipMemcpyHostToDevice, s0->stream) !=
                hipSuccess ||
            hipMemcpyAsync(R.state, state.data(), count * sizeof(BatchState), hipMemcpyHostToDevice, s0->stream) !=
                hipSuccess ||
            hipStreamSynchronize(s0->stream) != hipSuccess)
            return dev_fail("upload failed");
        for (size_t g = 1; g < spans.size(); ++g) {
            hipStream_t q = nullptr;
            if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) return dev_fail("stream creation failed");
            R.streams.push_back(q);
        }
        hipEvent_t fork = R.event(), t_a = R.event(), t_b = R.event();
        std::vector<hipEvent_t> join;
        for (size_t g = 1; g < spans.size(); ++g) join.push_back(R.event());
        if (!fork || !t_a || !t_b || std::find(join.begin(), join.end(), nullptr) != join.end())
            return dev_fail("event creation failed");
        // dynamic LDS beyond the default limit for the LX variants (a
        // runtime that needs no such opt-in may refuse the call: ignored)
        {
            const int most = (int)(kBatchLdsTotal - kBatchLdsStatic);
            if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<false, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, most) != hipSuccess ||
                hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<true, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, most) != hipSuccess)
                (void)hipGetLastError();
        }
        // capture: one branch per occupied group, a chain of launches each
        bool ok = hipStreamBeginCapture(s0->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            ok = hipEventRecord(fork, s0->stream) == hipSuccess;
            for (size_t g = 1; ok && g < spans.size(); ++g) ok = hipStreamWaitEvent(R.streams[g - 1], fork, 0) == hipSuccess;
            for (size_t g = 0; ok && g < spans.size(); ++g) {
                hipStream_t q = g ? R.streams[g - 1] : s0->stream;
                for (uint64_t done = 0; ok && done < nsteps;) {
                    const uint32_t chunk = (uint32_t)std::min<uint64_t>(kBatchChunk, nsteps - done);
                    // renumber every system in cell order before each chunk
                    hipLaunchKernelGGL(k_batch_sort, dim3(spans[g].second), dim3(threads[g]), 0, q,
                                       (const BatchItem*)(R.items + spans[g].first),
                                       (const BatchState*)(R.state + spans[g].first));
                    const BatchItem* it = R.items + spans[g].first;
                    BatchState* sg = R.state + spans[g].first;
                    const dim3 grid(spans[g].second), blk(threads[g]);
                    const size_t lds = xlds[g];
                    if (full[g] && lds)
                        hipLaunchKernelGGL((k_batch<true, true>), grid, blk, lds, q, it, sg, chunk);
                    else if (full[g])
                        hipLaunchKernelGGL((k_batch<true, false>), grid, blk, 0, q, it, sg, chunk);
                    else if (lds)
                        hipLaunchKernelGGL((k_batch<false, true>), grid, blk, lds, q, it, sg, chunk);
                    else
                        hipLaunchKernelGGL((k_batch<false, false>), grid, blk, 0, q, it, sg, chunk);
                    ok = hipGetLastError() == hipSuccess;
                    done += chunk;
                }
            }
            for (size_t g = 1; ok && g < spans.size(); ++g)
                ok = hipEventRecord(join[g - 1], R.streams[g - 1]) == hipSuccess &&
                     hipStreamWaitEvent(s0->stream, join[g - 1], 0) == hipSuccess;
            hipGraph_t graph = nullptr;
            const bool ended = hipStreamEndCapture(s0->stream, &graph) == hipSuccess;
            R.graph = graph;
            ok = ok && ended && graph;
        }
        if (!ok) {
            (void)hipGetLastError();
            return dev_fail("graph capture failed");
        }
        if (hipGraphInstantiate(&R.exec, R.graph, nullptr, nullptr, 0) != hipSuccess) return dev_fail("graph instantiation failed");
        if (hipEventRecord(t_a, s0->stream) != hipSuccess || hipGraphLaunch(R.exec, s0->stream) != hipSuccess ||
            hipEventRecord(t_b, s0->stream) != hipSuccess || hipStreamSynchronize(s0->stream) != hipSuccess)
            return dev_fail("launch failed");
        if (ms) (void)hipEventElapsedTime(ms, t_a, t_b);
    }
    for (uint32_t k = 0; k < count; ++k) {
        db_system* s = systems[k];
        s->step += nsteps;
        s->cur_x ^= (int)(nsteps & 1u);
        s->cur_list = (int)((s->cur_list + nsteps) % 3);
        s->tags_dirty = true;              // renumbered by k_batch_sort
    }
    for (uint32_t k = 0; k < count; ++k) {
        const db_status e = check_errors(systems[k]);
        if (e != DB_OK && st == DB_OK) st = e;
    }
    return st;
}

}  // namespace

extern "C" {

db_status db_step_batch_plan(db_system* const* systems, uint32_t count, uint64_t nsteps, const db_batch_plan* plan) {
    db_status st = batch_check(systems, count);
    if (st != DB_OK) return st;
    if (const char* why = plan_error(plan)) return fail(systems[0], DB_EINVAL, "%s", why);
    return run_batch(systems, count, nsteps, *plan, nullptr);
}

db_status db_step_batch(db_system* const* systems, uint32_t count, uint64_t nsteps) {
    db_status st = batch_check(systems, count);
    if (st != DB_OK) return st;
    db_batch_plan plan = default_plan();
    {
        std::lock_guard<std::mutex> lock(g_plan_mu);
        auto it = g_plans.find(systems[0]->device);
        if (it != g_plans.end()) plan = it->second;
    }
    return run_batch(systems, count, nsteps, plan, nullptr);
}

db_status db_set_batch_plan(int device, const db_batch_plan* plan) {
    if (plan && plan_error(plan)) return DB_EINVAL;
    if (!device_ok(device)) return DB_EDEVICE;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    if (plan) g_plans[device] = *plan;
    else g_plans.erase(device);
    return DB_OK;
}

db_status db_get_batch_plan(int device, db_batch_plan* plan) {
    if (!plan) return DB_EINVAL;
    if (!device_ok(device)) return DB_EDEVICE;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto it = g_plans.find(device);
    *plan = it != g_plans.end() ? it->second : default_plan();
    return DB_OK;
}

db_status db_batch_autotune(db_system* const* systems, uint32_t count, uint32_t trial_steps, db_batch_plan* best,
                            uint64_t* steps_done, double* trial_ms, uint32_t trial_len) {
    if (steps_done) *steps_done = 0;
    db_status st = batch_check(systems, count);
    if (st != DB_OK) return st;
    if (trial_steps < 1 || trial_steps > kBatchChunk)
        return fail(systems[0], DB_EINVAL, "trial_steps must be in [1, %u]", kBatchChunk);
    db_batch_plan p{};
    p.n_classes = 5;
    const uint32_t bounds[5] = {512u, 1024u, 2048u, 4096u, 0xFFFFFFFFu};
    for (uint32_t c = 0; c < 5; ++c) {
        p.n_max[c] = bounds[c];
        p.threads[c] = (uint32_t)kBatchMaxThreads;
    }
    bool occupied[5] = {};
    for (uint32_t k = 0; k < count; ++k) occupied[class_of(p, systems[k]->n)] = true;
    uint64_t done = 0;
    uint32_t nt = 0;
    auto trial = [&](const db_batch_plan& q, bool timed, float& ms) {
        const db_status e = run_batch(systems, count, trial_steps, q, timed ? &ms : nullptr);
        if (e == DB_OK || !systems[0]->dead) done += trial_steps;
        if (e == DB_OK && timed && trial_ms && nt < trial_len) trial_ms[nt] = ms;
        if (e == DB_OK && timed) ++nt;
        return e;
    };
    // Adjacent classes with the same workgroup size are merged: every class
    // is a graph branch of its own, and splitting a batch into branches that
    // gain nothing costs time (the largest systems of the whole batch no
    // longer start first): 5 classes of 1024 threads ran the sweep set 16 %
    // slower than one.
    auto merged = [](db_batch_plan q) {
        db_batch_plan r{};
        for (uint32_t c = 0; c < q.n_classes; ++c) {
            if (r.n_classes && r.threads[r.n_classes - 1] == q.threads[c]) {
                r.n_max[r.n_classes - 1] = q.n_max[c];
            } else {
                r.n_max[r.n_classes] = q.n_max[c];
                r.threads[r.n_classes] = q.threads[c];
                ++r.n_classes;
            }
        }
        return r;
    };
    // The systems move on from trial to trial (and the cost of a step with
    // them), so each candidate is judged against the plan in hand timed right
    // before and right after it: kept only if faster than both by 2 %.
    float t_prev = 0.0f, ms = 0.0f, t_after = 0.0f;
    st = trial(merged(p), false, ms);            // first run: code and caches warm up
    if (st == DB_OK) st = trial(merged(p), true, t_prev);
    const uint32_t cand[2] = {256u, 512u};
    for (uint32_t c = 0; c < 5 && st == DB_OK; ++c) {
        if (!occupied[c]) continue;
        for (uint32_t b : cand) {
            db_batch_plan q = p;
            q.threads[c] = b;
            st = trial(merged(q), true, ms);
            if (st == DB_OK) st = trial(merged(p), true, t_after);
            if (st != DB_OK) break;
            if (ms < 0.98f * std::min(t_prev, t_after)) {
                p = q;
                t_prev = ms;
            } else {
                t_prev = t_after;
            }
        }
    }
    if (steps_done) *steps_done = done;
    if (st != DB_OK) return st;
    p = merged(p);
    {
        std::lock_guard<std::mutex> lock(g_plan_mu);
        g_plans[systems[0]->device] = p;
    }
    if (best) *best = p;
    return DB_OK;
}

db_status db_sweep_frozen(db_system* s, uint64_t step_key) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (s->P.nrx == 0) return DB_OK;
    HIPCHK(s, hipSetDevice(s->device));
    const unsigned g = grid_of(s->n);
    const int xc = s->cur_x;
    LAUNCH(s, k_eval, g, kBlock, s->P, s->D, xc, 0u);
    const unsigned long long sv[2] = {step_key, step_key};
    const unsigned long long sv_back[2] = {s->step, s->step};
    HIPCHK(s, hipMemcpyAsync(s->D.stepv, sv, sizeof sv, hipMemcpyHostToDevice, s->stream));
    if (s->P.kt_kinetic) {
        HIPCHK(s, hipMemsetAsync(s->D.ke_fix, 0, 16, s->stream));
        LAUNCH(s, k_ke_accum, g, kBlock, s->P, s->D, xc, step_key);
    }
    launch_sweep(s, xc, (int)(step_key & 1));
    // both kinetic-energy slots start the next regular sweep cleared
    if (s->P.kt_kinetic) HIPCHK(s, hipMemsetAsync(s->D.ke_fix, 0, 16, s->stream));
    LAUNCH(s, k_eval, g, kBlock, s->P, s->D, xc, s->n);
    LAUNCH(s, k_fix_u, g, kBlock, s->P, s->D, xc);
    HIPCHK(s, hipMemcpyAsync(s->D.stepv, sv_back, sizeof sv_back, hipMemcpyHostToDevice, s->stream));
    return check_errors(s);
}

db_status db_set_state(db_system* s, uint64_t step, const float* pos3, const float* vel3,
                       const uint32_t* pairs, const uint32_t* bts, uint64_t m) {
    if (!s) return DB_EINVAL;
    if (s->dead) return fail(s, DB_EDEVICE, "device error earlier on this handle");
    if (!s->committed) return fail(s, DB_ESTATE, "system not committed");
    if (!pos3 || !vel3 || (m && (!pairs || !bts))) return fail(s, DB_EINVAL, "NULL arrays");
    db_status st = check_state(s, pos3, pairs, bts, m);
    if (st != DB_OK) return st;
    HIPCHK(s, hipSetDevice(s->device));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    st = ensure_cell_capacity(s, pos3);
    if (st != DB_OK) return st;
    s->step = step;
    return upload_state(s, pos3, vel3, pairs, bts, m);
}

db_status db_save_checkpoint(db_system* s, void* buf, uint64_t cap, uint64_t* size) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!size) return fail(s, DB_EINVAL, "size is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    const uint32_t n = s->n, nrx = (uint32_t)s->rx.size();
    const unsigned nb = grid_of(n);
    LAUNCH(s, k_rows_count, nb, kBlock, s->P, s->D, s->cur_x, s->bsum);
    LAUNCH(s, k_scan_bsum, 1, 1024, s->bsum, nb);
    uint32_t m = 0;
    HIPCHK(s, hipMemcpyAsync(&m, s->bsum + nb, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *size = ckpt_size(n, nrx, m);
    if (*size > cap) return fail(s, DB_ETRUNC, "checkpoint of %llu bytes, capacity %llu",
                                 (unsigned long long)*size, (unsigned long long)cap);
    if (!buf) return fail(s, DB_EINVAL, "buf is NULL");
    std::vector<uint32_t> pairs(2 * (size_t)m), bts(m);
    uint64_t m2 = 0;
    if (m) {
        st = db_read_bonds(s, pairs.data(), bts.data(), m, &m2);
        if (st != DB_OK) return st;
        if (m2 != m) return fail(s, DB_EDEVICE, "bond count changed during the checkpoint");
    }
    std::vector<float4> xh(n), uh(n);
    std::vector<int32_t> ih(3 * (size_t)n);
    std::vector<unsigned long long> slots((size_t)3 * kMaxRx * kCtrSlots);
    HIPCHK(s, hipMemcpyAsync(xh.data(), s->D.x[s->cur_x], n * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(uh.data(), s->D.u, n * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(ih.data(), s->D.img, ih.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(slots.data(), s->D.counters, slots.size() * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s->stream));
    st = check_errors(s);
    if (st != DB_OK) return st;
    st = sync_tags(s);
    if (st != DB_OK) return st;
    std::vector<uint64_t> ctr(3 * (size_t)nrx, 0);
    for (size_t c = 0; c < ctr.size(); ++c)
        for (uint32_t w = 0; w < kCtrSlots; ++w) ctr[c] += slots[c * kCtrSlots + w];
    std::vector<float> pos(3 * (size_t)n), vel(3 * (size_t)n);
    std::vector<int32_t> img(3 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i) {
        const size_t t = s->tag_h[i];
        pos[3 * t] = xh[i].x; pos[3 * t + 1] = xh[i].y; pos[3 * t + 2] = xh[i].z;
        vel[3 * t] = uh[i].x; vel[3 * t + 1] = uh[i].y; vel[3 * t + 2] = uh[i].z;
        for (uint32_t d = 0; d < 3; ++d) img[3 * t + d] = ih[(size_t)d * n + i];
    }
    unsigned char* o = (unsigned char*)buf + kCkptHeader;
    auto put = [&](const void* p, size_t k) { std::memcpy(o, p, k); o += k; };
    put(ctr.data(), ctr.size() * 8);
    put(pos.data(), pos.size() * 4);
    put(vel.data(), vel.size() * 4);
    put(img.data(), img.size() * 4);
    put(pairs.data(), pairs.size() * 4);
    put(bts.data(), bts.size() * 4);
    Fnv ph;
    ph.bytes((const unsigned char*)buf + kCkptHeader, *size - kCkptHeader);
    unsigned char* h = (unsigned char*)buf;
    const uint32_t hw[4] = {kCkptMagic, kCkptVersion, n, nrx};
    const uint64_t hq[4] = {s->step, (uint64_t)m, config_fingerprint(s), ph.h};
    std::memcpy(h, hw, sizeof hw);
    std::memcpy(h + sizeof hw, hq, sizeof hq);
    return DB_OK;
}

db_status db_load_checkpoint(db_system* s, const void* buf, uint64_t size) {
    if (!s) return DB_EINVAL;
    if (s->dead) return fail(s, DB_EDEVICE, "device error earlier on this handle");
    if (!s->committed) return fail(s, DB_ESTATE, "system not committed");
    if (!buf) return fail(s, DB_EINVAL, "buf is NULL");
    if (size < kCkptHeader) return fail(s, DB_EINVAL, "checkpoint shorter than its header");
    uint32_t hw[4];
    uint64_t hq[4];
    std::memcpy(hw, buf, sizeof hw);
    std::memcpy(hq, (const unsigned char*)buf + sizeof hw, sizeof hq);
    if (hw[0] != kCkptMagic) return fail(s, DB_EINVAL, "not a checkpoint");
    if (hw[1] != kCkptVersion) return fail(s, DB_EINVAL, "checkpoint version %u, expected %u", hw[1], kCkptVersion);
    const uint32_t n = s->n, nrx = (uint32_t)s->rx.size();
    if (hw[2] != n || hw[3] != nrx)
        return fail(s, DB_EINVAL, "checkpoint of %u particles and %u reactions, system has %u and %u", hw[2], hw[3], n, nrx);
    const uint64_t m = hq[1];
    if (m > (uint64_t)n * kMaxValence || size != ckpt_size(n, nrx, m))
        return fail(s, DB_EINVAL, "checkpoint size %llu does not match its header", (unsigned long long)size);
    if (hq[2] != config_fingerprint(s))
        return fail(s, DB_EINVAL, "checkpoint of a system set up differently (types, bonds, reactions, integrator)");
    Fnv ph;
    ph.bytes((const unsigned char*)buf + kCkptHeader, size - kCkptHeader);
    if (ph.h != hq[3]) return fail(s, DB_EINVAL, "checkpoint payload damaged (hash mismatch)");
    const unsigned char* c = (const unsigned char*)buf + kCkptHeader;
    auto take = [&](void* p, size_t k) { std::memcpy(p, c, k); c += k; };
    std::vector<uint64_t> ctr(3 * (size_t)nrx);
    std::vector<float> pos(3 * (size_t)n), vel(3 * (size_t)n);
    std::vector<int32_t> img(3 * (size_t)n);
    std::vector<uint32_t> pairs(2 * (size_t)m), bts(m);
    take(ctr.data(), ctr.size() * 8);
    take(pos.data(), pos.size() * 4);
    take(vel.data(), vel.size() * 4);
    take(img.data(), img.size() * 4);
    take(pairs.data(), pairs.size() * 4);
    take(bts.data(), bts.size() * 4);
    db_status st = check_state(s, pos.data(), pairs.data(), bts.data(), m);
    if (st != DB_OK) return st;
    HIPCHK(s, hipSetDevice(s->device));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    st = ensure_cell_capacity(s, pos.data());
    if (st != DB_OK) return st;
    const uint64_t step_before = s->step;
    s->step = hq[0];
    st = upload_state(s, pos.data(), vel.data(), pairs.data(), bts.data(), m, true, img.data());
    if (st != DB_OK) { s->step = step_before; return st; }
    // cumulative counters: each total in the first slot of its spread
    std::vector<unsigned long long> slots((size_t)3 * kMaxRx * kCtrSlots, 0ull);
    for (size_t k = 0; k < ctr.size(); ++k) slots[k * kCtrSlots] = ctr[k];
    HIPCHK(s, hipMemcpyAsync(s->D.counters, slots.data(), slots.size() * sizeof(unsigned long long),
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return DB_OK;
}

// Before db_commit the read-outs of positions and velocities return the
// set-up state (host copies; no GPU is touched).
static db_status read_setup(db_system* s, float* out3, bool velocities, int32_t* image3) {
    if (!out3) return fail(s, DB_EINVAL, "output is NULL");
    if (!s->have_particles) return fail(s, DB_ESTATE, "particles not set");
    if (velocities && !s->vel_given && !s->validated)
        return fail(s, DB_ESTATE, "velocities not given: they are drawn by db_validate");
    const std::vector<float>& src = velocities ? s->vel : s->pos;
    std::memcpy(out3, src.data(), 3 * (size_t)s->n * sizeof(float));
    if (image3) std::memset(image3, 0, 3 * (size_t)s->n * sizeof(int32_t));
    return DB_OK;
}

db_status db_read_positions(db_system* s, float* pos3, int32_t* image3) {
    if (s && !s->committed && !s->dead) return read_setup(s, pos3, false, image3);
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!pos3) return fail(s, DB_EINVAL, "pos3 is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    LAUNCH(s, k_gather, grid_of(s->n), kBlock, s->P, s->D, s->stage, s->cur_x, 0);
    std::vector<float4> h(s->n);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->stage, s->n * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    std::vector<int32_t> im;
    if (image3) {
        // the staging buffer (16 n bytes) is reused for 12 n bytes of image counters;
        // the position copy above is ordered before this kernel on the stream
        LAUNCH(s, k_gather_img, grid_of(s->n), kBlock, s->P, s->D, (int32_t*)s->stage);
        im.resize(3 * (size_t)s->n);
        HIPCHK(s, hipMemcpyAsync(im.data(), s->stage, im.size() * 4, hipMemcpyDeviceToHost, s->stream));
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (uint32_t t = 0; t < s->n; ++t) {
        pos3[3 * t] = h[t].x;
        pos3[3 * t + 1] = h[t].y;
        pos3[3 * t + 2] = h[t].z;
    }
    if (image3) std::memcpy(image3, im.data(), im.size() * 4);
    return DB_OK;
}

static db_status read_vec(db_system* s, float* out3, int mode) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!out3) return fail(s, DB_EINVAL, "output is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    LAUNCH(s, k_eval, grid_of(s->n), kBlock, s->P, s->D, s->cur_x, 0u);
    LAUNCH(s, k_gather, grid_of(s->n), kBlock, s->P, s->D, s->stage, s->cur_x, mode);
    std::vector<float4> h(s->n);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->stage, s->n * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    st = check_errors(s);
    if (st != DB_OK) return st;
    for (uint32_t t = 0; t < s->n; ++t) {
        out3[3 * t] = h[t].x;
        out3[3 * t + 1] = h[t].y;
        out3[3 * t + 2] = h[t].z;
    }
    return DB_OK;
}

// Device-side read-out on the caller's stream, ordered after the system's
// pending work, with the system's later work ordered after it.
static db_status read_vec_device(db_system* s, float* out3, void* stream, int mode) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!out3) return fail(s, DB_EINVAL, "output is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    const hipStream_t q = stream ? (hipStream_t)stream : s->stream;
    if (mode != 0) LAUNCH(s, k_eval, grid_of(s->n), kBlock, s->P, s->D, s->cur_x, 0u);
    if (q != s->stream) {
        if (!s->ev_out) HIPCHK(s, hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
        if (!s->ev_back) HIPCHK(s, hipEventCreateWithFlags(&s->ev_back, hipEventDisableTiming));
        HIPCHK(s, hipEventRecord(s->ev_out, s->stream));
        HIPCHK(s, hipStreamWaitEvent(q, s->ev_out, 0));
    }
    hipLaunchKernelGGL(k_gather3, dim3(grid_of(s->n)), dim3(kBlock), 0, q, s->P, s->D, out3, s->cur_x, mode);
    HIPCHK(s, hipGetLastError());
    if (q != s->stream) {
        HIPCHK(s, hipEventRecord(s->ev_back, q));
        HIPCHK(s, hipStreamWaitEvent(s->stream, s->ev_back, 0));
    }
    return DB_OK;
}

db_status db_read_positions_device(db_system* s, float* pos3, void* stream) { return read_vec_device(s, pos3, stream, 0); }
db_status db_read_velocities_device(db_system* s, float* vel3, void* stream) { return read_vec_device(s, vel3, stream, 1); }
db_status db_read_forces_device(db_system* s, float* force3, void* stream) { return read_vec_device(s, force3, stream, 2); }

db_status db_read_velocities(db_system* s, float* vel3) {
    if (s && !s->committed && !s->dead) return read_setup(s, vel3, true, nullptr);
    return read_vec(s, vel3, 1);
}
db_status db_read_forces(db_system* s, float* force3) { return read_vec(s, force3, 2); }

db_status db_read_bonds(db_system* s, uint32_t* pairs, uint32_t* bts, uint64_t cap, uint64_t* count) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!count) return fail(s, DB_EINVAL, "count is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    const unsigned nb = grid_of(s->n);
    LAUNCH(s, k_rows_count, nb, kBlock, s->P, s->D, s->cur_x, s->bsum);
    LAUNCH(s, k_scan_bsum, 1, 1024, s->bsum, nb);
    uint32_t total = 0;
    HIPCHK(s, hipMemcpyAsync(&total, s->bsum + nb, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *count = total;
    if (total > cap) return fail(s, DB_ETRUNC, "%u bonds, capacity %llu", total, (unsigned long long)cap);
    if (total == 0) return DB_OK;
    if (!pairs || !bts) return fail(s, DB_EINVAL, "NULL output arrays");
    uint32_t *dp = nullptr, *db = nullptr;
    HIPCHK(s, hipMallocAsync((void**)&dp, (size_t)total * 8, s->stream));
    HIPCHK(s, hipMallocAsync((void**)&db, (size_t)total * 4, s->stream));
    LAUNCH(s, k_rows_emit, nb, kBlock, s->P, s->D, s->cur_x, s->bsum, dp, db);
    HIPCHK(s, hipMemcpyAsync(pairs, dp, (size_t)total * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(bts, db, (size_t)total * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipFreeAsync(dp, s->stream));
    HIPCHK(s, hipFreeAsync(db, s->stream));
    return check_errors(s);
}

// Device address of `scratch` on each device, looked up once per device
// (with that device current) on the first db_read_bonds_noalloc call there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch[kMaxDevices] = {};

static db_status scratch_on(db_system* s, uint32_t** out) {
    if (s->device < 0 || s->device >= kMaxDevices) return fail(s, DB_EDEVICE, "device %d out of range", s->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[s->device]) {
        void* p = nullptr;
        HIPCHK(s, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[s->device] = (uint32_t*)p;
    }
    *out = g_scratch[s->device];
    return DB_OK;
}

db_status db_read_bonds_noalloc(db_system* s, uint32_t* pairs, uint32_t* bts, uint64_t cap, uint64_t* count) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!count) return fail(s, DB_EINVAL, "count is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    uint32_t* sp = nullptr;
    st = scratch_on(s, &sp);
    if (st != DB_OK) return st;
    const unsigned nb = grid_of(s->n);
    LAUNCH(s, k_rows_count, nb, kBlock, s->P, s->D, s->cur_x, s->bsum);
    LAUNCH(s, k_scan_bsum, 1, 1024, s->bsum, nb);
    uint32_t total = 0;
    HIPCHK(s, hipMemcpyAsync(&total, s->bsum + nb, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *count = total;
    if (total > cap) return fail(s, DB_ETRUNC, "%u bonds, capacity %llu", total, (unsigned long long)cap);
    if (total > kNoAllocBonds)
        return fail(s, DB_ENOMEM, "%u bonds exceed the %u of the fixed staging array (use db_read_bonds)", total,
                    kNoAllocBonds);
    if (total == 0) return DB_OK;
    if (!pairs || !bts) return fail(s, DB_EINVAL, "NULL output arrays");
    uint32_t* const dp = sp;                      // tag pairs
    uint32_t* const dt = sp + 2 * (size_t)kNoAllocBonds;   // bond types
    LAUNCH(s, k_rows_emit, nb, kBlock, s->P, s->D, s->cur_x, s->bsum, dp, dt);
    HIPCHK(s, hipMemcpyAsync(pairs, dp, (size_t)total * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(bts, dt, (size_t)total * 4, hipMemcpyDeviceToHost, s->stream));
    return check_errors(s);
}

db_status db_read_sweep_events(db_system* s, int which, uint32_t* pairs, uint32_t* bts, uint64_t cap,
                               uint64_t* count, uint64_t* sweep_step) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!count) return fail(s, DB_EINVAL, "count is NULL");
    if (which != DB_EVENT_FORMED && which != DB_EVENT_BROKEN)
        return fail(s, DB_EINVAL, "which must be DB_EVENT_FORMED or DB_EVENT_BROKEN");
    HIPCHK(s, hipSetDevice(s->device));
    uint32_t c[4];
    HIPCHK(s, hipMemcpyAsync(c, s->D.evc, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const uint32_t m = c[which];
    if (m > s->P.evcap[which]) return fail(s, DB_EDEVICE, "event list longer than its bound (%u > %u)", m, s->P.evcap[which]);
    *count = m;
    if (sweep_step) *sweep_step = ((uint64_t)c[3] << 32) | c[2];
    if (m > cap) return fail(s, DB_ETRUNC, "%u events, capacity %llu", m, (unsigned long long)cap);
    if (m == 0) return DB_OK;
    if (!pairs || !bts) return fail(s, DB_EINVAL, "NULL output arrays");
    std::vector<uint2> e(m);
    HIPCHK(s, hipMemcpyAsync(e.data(), s->D.ev[which], (size_t)m * sizeof(uint2), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    std::vector<std::array<uint32_t, 3>> rows(m);
    for (uint32_t k = 0; k < m; ++k) {
        const uint32_t a = e[k].y >> 24;
        if (a >= s->P.nrx) return fail(s, DB_EDEVICE, "event with reaction %u", a);
        rows[k] = {e[k].x, e[k].y & kIdxMask, s->P.rbt[a]};
    }
    std::sort(rows.begin(), rows.end());
    for (uint32_t k = 0; k < m; ++k) {
        pairs[2 * k] = rows[k][0];
        pairs[2 * k + 1] = rows[k][1];
        bts[k] = rows[k][2];
    }
    return check_errors(s);
}

// Clusters of static + dynamic bonds: union by minimum index until no hook
// changes a root; then D.parent holds each particle's root and D.scan each
// root's cluster size.
static db_status label_clusters(db_system* s) {
    const unsigned g = grid_of(s->n);
    const Params& P = s->P;
    LAUNCH(s, k_cc_init, g, kBlock, P, s->D);
    for (int it = 0; it < 64; ++it) {
        uint32_t changed = 0;
        HIPCHK(s, hipMemsetAsync(s->flag, 0, 4, s->stream));
        LAUNCH(s, k_cc_hook, g, kBlock, P, s->D, s->flag, s->cur_x);
        LAUNCH(s, k_cc_compress, g, kBlock, P, s->D);
        HIPCHK(s, hipMemcpyAsync(&changed, s->flag, 4, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        if (!changed) break;
        if (it == 63) return fail(s, DB_EDEVICE, "cluster labelling did not converge");
    }
    HIPCHK(s, hipMemsetAsync(s->D.scan, 0, (size_t)s->n * 4, s->stream));
    LAUNCH(s, k_cc_size, g, kBlock, P, s->D);
    return DB_OK;
}

db_status db_cluster_sizes(db_system* s, uint64_t* hist, uint32_t len, uint64_t* n_clusters) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!hist || !n_clusters || len < 1 || len > kAnaHist)
        return fail(s, DB_EINVAL, "histogram of 1..%u bins and output pointers required", kAnaHist);
    HIPCHK(s, hipSetDevice(s->device));
    st = label_clusters(s);
    if (st != DB_OK) return st;
    HIPCHK(s, hipMemsetAsync(s->ana, 0, kAnaWords * 8, s->stream));
    LAUNCH(s, k_cc_hist, grid_of(s->n), kBlock, s->P, s->D, s->ana + 1, len, s->ana);
    unsigned long long h[kAnaWords];
    HIPCHK(s, hipMemcpyAsync(h, s->ana, (len + 1) * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *n_clusters = h[0];
    for (uint32_t k = 0; k < len; ++k) hist[k] = h[1 + k];
    return check_errors(s);
}

db_status db_bond_reference(db_system* s) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    HIPCHK(s, hipSetDevice(s->device));
    if (!s->bref) DALLOC(s, s->bref, (size_t)std::max(s->P.cap_max, 1u) * s->n);
    LAUNCH(s, k_bond_ref, grid_of(s->n), kBlock, s->P, s->D, s->bref, s->cur_x);
    HIPCHK(s, hipGetLastError());
    s->have_ref = true;
    return DB_OK;
}

db_status db_bond_correlation(db_system* s, uint64_t* n_reference, uint64_t* n_intact) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!n_reference || !n_intact) return fail(s, DB_EINVAL, "NULL outputs");
    if (!s->have_ref) return fail(s, DB_ESTATE, "no reference bonds (call db_bond_reference first)");
    HIPCHK(s, hipSetDevice(s->device));
    HIPCHK(s, hipMemsetAsync(s->ana, 0, 16, s->stream));
    LAUNCH(s, k_bond_corr, grid_of(s->n), kBlock, s->P, s->D, s->bref, s->ana);
    unsigned long long h[2];
    HIPCHK(s, hipMemcpyAsync(h, s->ana, 16, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *n_reference = h[0];
    *n_intact = h[1];
    return check_errors(s);
}

db_status db_bond_multiplicity(db_system* s, uint64_t* hist, uint32_t len, uint64_t* n_pairs, uint64_t* n_intra) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!hist || !n_pairs || !n_intra || len < 1 || len > kAnaHist)
        return fail(s, DB_EINVAL, "histogram of 1..%u bins and output pointers required", kAnaHist);
    HIPCHK(s, hipSetDevice(s->device));
    // table: a power of two at least twice the largest possible number of bonds
    uint64_t max_bonds = 0;
    for (uint32_t i = 0; i < s->n; ++i) max_bonds += s->types[s->type[i]].valence;
    uint32_t size = 1024;
    while (size < 2 * (max_bonds / 2 + 1)) size *= 2;
    unsigned long long* keys = nullptr;
    uint32_t* counts = nullptr;
    HIPCHK(s, hipMallocAsync((void**)&keys, (size_t)size * 8, s->stream));
    HIPCHK(s, hipMallocAsync((void**)&counts, (size_t)size * 4, s->stream));
    HIPCHK(s, hipMemsetAsync(keys, 0xFF, (size_t)size * 8, s->stream));
    HIPCHK(s, hipMemsetAsync(counts, 0, (size_t)size * 4, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ana, 0, kAnaWords * 8, s->stream));
    LAUNCH(s, k_mol_pairs, grid_of(s->n), kBlock, s->P, s->D, s->cur_x, keys, counts, size - 1u, s->ana);
    LAUNCH(s, k_mol_hist, grid_of(size), kBlock, keys, counts, size, s->ana + 2, len, s->ana + 1);
    unsigned long long h[kAnaWords];
    HIPCHK(s, hipMemcpyAsync(h, s->ana, (len + 2) * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipFreeAsync(keys, s->stream));
    HIPCHK(s, hipFreeAsync(counts, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *n_intra = h[0];
    *n_pairs = h[1];
    for (uint32_t k = 0; k < len; ++k) hist[k] = h[2 + k];
    return check_errors(s);
}

db_status db_read_observables(db_system* s, db_observables* out) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!out) return fail(s, DB_EINVAL, "out is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    const unsigned g = grid_of(s->n);
    const Params& P = s->P;
    LAUNCH(s, k_eval, g, kBlock, P, s->D, s->cur_x, 0u);
    HIPCHK(s, hipMemsetAsync(s->D.red, 0, (4 + kMaxRx) * 8, s->stream));
    LAUNCH(s, k_observe, g, kBlock, P, s->D, s->cur_x);
    // largest cluster
    st = label_clusters(s);
    if (st != DB_OK) return st;
    LAUNCH(s, k_cc_max, g, kBlock, P, s->D);
    unsigned long long red[4 + kMaxRx];
    std::vector<unsigned long long> slots((size_t)3 * kMaxRx * kCtrSlots);
    HIPCHK(s, hipMemcpyAsync(red, s->D.red, sizeof red, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(slots.data(), s->D.counters, slots.size() * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s->stream));
    st = check_errors(s);
    if (st != DB_OK) return st;
    unsigned long long ctr[3 * kMaxRx] = {};
    for (size_t c = 0; c < (size_t)3 * kMaxRx; ++c)
        for (uint32_t w = 0; w < kCtrSlots; ++w) ctr[c] += slots[c * kCtrSlots + w];
    std::memset(out, 0, sizeof *out);
    out->step = s->step;
    out->n_reactions = P.nrx;
    out->pe = (double)red[0] * kFixInv;
    out->ke = (double)red[1] * kFixInv;
    out->t_kin = 2.0 * out->ke / (3.0 * (double)s->n);
    out->largest_cluster_fraction = (double)red[2 + kMaxRx] / (double)s->n;
    for (uint32_t a = 0; a < P.nrx; ++a) {
        out->n_bonds[a] = red[2 + a];
        out->attempts[a] = ctr[3 * a];
        out->forms[a] = ctr[3 * a + 1];
        out->breaks[a] = ctr[3 * a + 2];
        double cap_a = 0, cap_b = 0;
        for (uint32_t i = 0; i < s->n; ++i) {
            if (s->type[i] == s->rx[a].type_a) cap_a += s->types[s->type[i]].valence;
            if (s->type[i] == s->rx[a].type_b) cap_b += s->types[s->type[i]].valence;
        }
        const double denom = s->rx[a].type_a == s->rx[a].type_b ? cap_a / 2.0 : std::min(cap_a, cap_b);
        out->bonded_fraction[a] = denom > 0 ? (double)red[2 + a] / denom : 0.0;
    }
    return DB_OK;
}

uint64_t db_get_step(const db_system* s) { return s ? s->step : 0; }

db_status db_read_list_builds(db_system* s, uint64_t* builds) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    if (!builds) return fail(s, DB_EINVAL, "builds is NULL");
    HIPCHK(s, hipSetDevice(s->device));
    uint32_t c = 0;
    HIPCHK(s, hipMemcpyAsync(&c, s->D.rflag + 4, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *builds = c;
    return DB_OK;
}

const char* db_last_error(const db_system* s) { return s ? s->err.c_str() : g_create_error.c_str(); }

db_status db_set_stream(db_system* s, void* stream) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    destroy_graphs(s);
    s->stream = stream ? (hipStream_t)stream : s->own_stream;
    return DB_OK;
}

db_status db_kernel_timing(db_system* s, int enable) {
    db_status st = ready(s);
    if (st != DB_OK) return st;
    flush_timing(s);
    s->timing.on = enable != 0;
    if (enable) s->timing.acc.clear();
    return DB_OK;
}

db_status db_read_kernel_time(db_system* s, const char* kernel, uint64_t* launches, double* total_ms) {
    if (!s || !kernel) return DB_EINVAL;
    flush_timing(s);
    auto it = s->timing.acc.find(kernel);
    if (launches) *launches = it == s->timing.acc.end() ? 0 : it->second.first;
    if (total_ms) *total_ms = it == s->timing.acc.end() ? 0.0 : it->second.second;
    return DB_OK;
}

}  // extern "C"
