// Host side of the CR-MC library: the C ABI declared in include/crmc.h.
//
// Holds per-replica geometry, converts positions to the fixed-point lattice,
// performs the initial stable binning into the unshifted grid, allocates the
// device buffers, turns reservoir conditions into the log acceptance
// constants of Sec. II C (FP64) and enqueues the sweep kernels.
#include "crmc.h"
#include "crmc_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace crmc;

namespace {

constexpr double TWO32 = 4294967296.0;
constexpr double LN10 = 2.302585092994045684017991454684364208;
constexpr int DEFAULT_POOL = 4096;          // LDS pool per phase workgroup (records, 64 KB)
constexpr int64_t DEFAULT_SERIES = 16384;   // retained sweeps of the series

struct HostReplica {
    bool built = false;
    double L = 0.0;
    uint32_t n = 0, cap = 0, ncells = 0, ncores = 0, nsites = 0, ngroups = 0;
    uint32_t site_bound = 0;  // most non-ion particles any shifted cell can hold
    int64_t nA = 0, nB = 0;
    double E0 = 0.0;          // energy at the last restart of the running sum
    double e0_kappa = 0.0;    // screening length E0 was computed with (NaN: not yet)
    std::vector<int32_t> hist_off;
    crmc_cond cond{};
    Replica d{}; // device pointers and constants (host copy of the descriptor)
    // The initial state as built, kept on the host until the first call that
    // needs the device state (so that a workspace can still be attached):
    // records in cell order, cell counts, per-site groups, cores.
    bool on_device = false;
    double* md_vel[2] = {nullptr, nullptr}; // molecular dynamics: 3 doubles per record slot per buffer
    double* md_force = nullptr;
    std::vector<uint4> init_rec;
    std::vector<uint32_t> init_cnt;
    std::vector<int32_t> init_group;
    std::vector<uint4> init_cores;
    std::vector<double> init_delta;
    int64_t init_tot[4] = {0, 0, 0, 0};
    uint32_t init_maxc = 0;
    int64_t n_built = 0;   // particles the replica was built with
};

// Device memory of a handle: the library's own allocations, or blocks of a
// caller-owned workspace handed out first fit (256-byte aligned) and given
// back on release, neighbouring free blocks merged.
constexpr size_t WS_ALIGN = 256;

size_t ws_round(size_t b) { return (std::max<size_t>(b, 1) + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_blocks; // offset -> bytes
    std::map<const void*, size_t> live;   // pointer -> bytes
    size_t used = 0;

    void attach(void* p, size_t bytes)
    {
        const uintptr_t a = ((uintptr_t)p + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
        const size_t lost = (size_t)(a - (uintptr_t)p);
        base = (char*)a;
        size = bytes > lost ? (bytes - lost) / WS_ALIGN * WS_ALIGN : 0;
        free_blocks.clear();
        live.clear();
        used = 0;
        if (size) free_blocks[0] = size;
    }
    void* take(size_t bytes)
    {
        bytes = ws_round(bytes);
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_blocks.erase(it);
            if (rest) free_blocks[off + bytes] = rest;
            void* q = base + off;
            live[q] = bytes;
            used += bytes;
            return q;
        }
        return nullptr;
    }
    bool give(const void* q)
    {
        auto it = live.find(q);
        if (it == live.end()) return false;
        size_t off = (size_t)((const char*)q - base), bytes = it->second;
        live.erase(it);
        used -= bytes;
        auto nx = free_blocks.lower_bound(off);
        if (nx != free_blocks.end() && nx->first == off + bytes) {
            bytes += nx->second;
            nx = free_blocks.erase(nx);
        }
        if (nx != free_blocks.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return true;
            }
        }
        free_blocks[off] = bytes;
        return true;
    }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto& kv : free_blocks) m = std::max(m, kv.second);
        return m;
    }
};

} // namespace

struct crmc_s {
    crmc_params p{};
    std::vector<HostReplica> reps;
    Arena ws;                    // caller-owned workspace (ws.base null: the library allocates)
    bool device_state = false;   // some device memory of the handle exists
    std::map<const void*, size_t> own; // the library's own live allocations (bytes, rounded)
    Replica* d_reps = nullptr;
    uint32_t* d_cell2rep = nullptr;
    uint32_t* d_dom2rep = nullptr;
    double* d_lntab = nullptr;
    int32_t lntab_n = 0;
    uint32_t ncell_total = 0, ndom_total = 0;
    uint64_t* d_sweep = nullptr;
    uint32_t* d_err = nullptr;
    uint32_t* d_plan_n = nullptr;     // per colour: heavy and light domain counts
    uint32_t* d_plan_heavy = nullptr; // per colour: ndom_total domain slots
    uint32_t* d_plan_light = nullptr;
    uint4* d_plan_geo_heavy = nullptr;  // beside each slot: replica, cells, counts
    uint4* d_plan_geo_light = nullptr;
    // learned proposal
    bool learned = false;
    double learn_eps = 0.1;
    uint64_t* d_R2sh = nullptr;      // 17 shell thresholds per replica
    float* d_p32 = nullptr;          // FP32 master parameters
    double* d_p64 = nullptr;
    short* d_w1b = nullptr;
    short* d_w2b = nullptr;
    float* d_adam_m = nullptr;
    float* d_adam_v = nullptr;
    float* d_grad = nullptr;
    double* d_loss = nullptr;
    int64_t adam_t = 0;
    float* d_data = nullptr;         // training rows (32 features + label)
    unsigned long long* d_data_n = nullptr;
    int64_t data_cap = 0;
    bool collecting = false;
    bool learn_lds_set = false;
    int ncu = 0;                     // compute units of the device
    LearnItem* d_lwork = nullptr;    // per colour: work items of the feature kernel
    uint32_t lwork_cap = 0;
    TrialRec* d_log = nullptr;
    unsigned long long* d_log_n = nullptr;
    int64_t log_cap = 0;
    PhaseTrace* d_trace = nullptr;
    unsigned long long* d_trace_n = nullptr;
    int64_t trace_cap = 0;
    int64_t sweeps = 0;
    int pool = DEFAULT_POOL;
    size_t lds_attr = 0; // dynamic LDS the phase kernel is currently allowed
    hipStream_t stream = nullptr;
    std::string err;
    // kernel timing
    bool timing = false;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    double t_ms[3] = {0, 0, 0};
    int64_t t_n[3] = {0, 0, 0};
    // captured sweeps: [0] one sweep, [1] GRAPH_SWEEPS sweeps
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<uint8_t> gargs; // launch arguments the captured graphs were recorded with
    // molecular dynamics: steps run so far (counter of their random numbers), pointer tables
    uint64_t md_steps = 0;
    double** d_md_vel = nullptr;   // 2 per replica
    double** d_md_force = nullptr; // 1 per replica
    // recorded per-site features (checks of the learned proposal)
    bool record_feat = false;
};

namespace {

int fail(crmc_t h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    return code;
}

#define HIP_TRY(h, expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), e_ == hipErrorOutOfMemory ? CRMC_E_NOMEM : CRMC_E_DEVICE,      \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

uint64_t cutoff_R2(double rc, double L)
{
    const double t = (rc / L) * TWO32;
    return (uint64_t)std::ceil(t * t);
}

uint32_t to_fixed(double x, double L)
{
    double f = x / L;
    f -= std::floor(f);
    double v = std::floor(f * TWO32);
    if (v >= TWO32) v = 0.0;
    return (uint32_t)v;
}

uint64_t cell_lo_h(uint32_t k, uint32_t n) { return (((uint64_t)k << 32) + n - 1u) / n; }
uint32_t cell_of_h(uint32_t y, uint32_t n) { return (uint32_t)(((uint64_t)y * n) >> 32); }

// cells two apart never interact: a full cell lies between them
bool grid_ok(uint32_t n, uint64_t R2)
{
    if (n < 4 || (n & 1u)) return false;
    const uint64_t wmin = (uint64_t)(TWO32 / n); // floor(2^32 / n)
    const uint64_t sep = wmin + 1u;
    return sep * sep >= R2;
}

// device memory for count values of T: from the workspace when one is
// attached (hipErrorOutOfMemory when it has no block that large), else from
// the runtime
template <typename T>
hipError_t dalloc(crmc_t h, T** p, size_t count)
{
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    h->device_state = true;
    if (h->ws.base) {
        *p = (T*)h->ws.take(bytes);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    const hipError_t e = hipMalloc((void**)p, bytes);
    if (e == hipSuccess) h->own[*p] = ws_round(bytes);
    return e;
}

void dfree(crmc_t h, void* q)
{
    if (!q) return;
    if (h->ws.base && h->ws.give(q)) return;
    h->own.erase(q);
    (void)hipFree(q);
}

void free_replica(crmc_t h, HostReplica& r)
{
    Replica& d = r.d;
    void* ptrs[] = {d.rec[0], d.rec[1], d.cnt[0], d.cnt[1], d.cnt0, d.e_acc, d.occupancy, d.site_group,
                    d.group_count, d.group_hist, d.group_hist_off, d.core_x, d.core_delta, d.totals,
                    d.moves, d.ctr, d.series, d.bnd, d.lnW, d.hiwater, d.tab, d.phat, d.nsc, d.feat};
    for (void* q : ptrs) dfree(h, q);
    for (double*& q : r.md_vel) { dfree(h, q); q = nullptr; }
    dfree(h, r.md_force);
    r.md_force = nullptr;
    d = Replica{};
    r.built = false;
    r.on_device = false;
}

void set_conditions(crmc_t h, HostReplica& r, const crmc_cond& c)
{
    r.cond = c;
    const double pOH = h->p.pKw - c.pH;
    r.d.lnKA = (c.pH - c.pKa - c.pIX_pos) * LN10;
    r.d.lnKB = (pOH - c.pKb - c.pIX_neg) * LN10;
    r.d.lnKion = -(c.pIX_pos + c.pIX_neg) * LN10;
    r.d.kappa = c.kappa;
}

SweepArgs base_args(crmc_t h)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.reps = h->d_reps;
    a.cell2rep = h->d_cell2rep;
    a.dom2rep = h->d_dom2rep;
    a.lntab = h->d_lntab;
    a.lntab_n = h->lntab_n;
    a.ln2 = std::log(2.0);
    a.nrep = (uint32_t)h->reps.size();
    a.ncell_total = h->ncell_total;
    a.ndom_total = h->ndom_total;
    a.sweep = h->d_sweep;
    a.err = h->d_err;
    a.log = h->d_log;
    a.log_n = h->d_log_n;
    a.log_cap = (uint64_t)h->log_cap;
    a.lB = h->p.lB;
    a.eps = h->p.eps_wca;
    a.ion_coupling = h->p.ion_coupling;
    a.trials = h->p.trials_per_cell;
    a.pairing = h->p.pairing;
    a.fixed_grid = h->p.fixed_grid;
    a.site_trials = h->p.site_trials;
    a.ion_trials = h->p.ion_trials;
    a.bin_sparse_any = 0;
    a.bin_dense_any = 0;
    for (const auto& r : h->reps) {
        a.bin_sparse_any |= (int32_t)r.d.bin_sparse;
        a.bin_dense_any |= (int32_t)!r.d.bin_sparse;
    }
    a.bin_cpw = a.ncell_total >= BIN_BATCH_MIN_CELLS ? (int32_t)BIN_CPW : 1;
    a.pool = h->pool;
    a.precision = h->p.precision;
    a.light_nb = h->p.light_neighbours > 0 ? h->p.light_neighbours : DEFAULT_LIGHT_NB;
    a.plan_n = h->d_plan_n;
    a.plan_heavy = h->d_plan_heavy;
    a.plan_light = h->d_plan_light;
    a.plan_geo_heavy = h->d_plan_geo_heavy;
    a.plan_geo_light = h->d_plan_geo_light;
    a.learned = h->learned ? 1 : 0;
    a.learn_eps = h->learn_eps;
    a.trace = h->d_trace;
    a.trace_n = h->d_trace_n;
    a.trace_cap = (uint64_t)h->trace_cap;
    return a;
}

int upload_descriptors(crmc_t h)
{
    std::vector<Replica> v(h->reps.size());
    uint32_t cells = 0, doms = 0;
    for (size_t i = 0; i < h->reps.size(); ++i) {
        HostReplica& r = h->reps[i];
        // the re-binning takes BIN_CPW cells of one replica per wavefront
        if (r.ncells % BIN_CPW != 0) return fail(h, CRMC_E_DEVICE, "internal error: cell count not a multiple of eight");
        r.d.cell_begin = cells;
        r.d.dom_begin = doms;
        cells += r.ncells;
        const uint32_t M = r.d.h * r.d.h * r.d.h;
        doms += h->p.pairing ? (M + 1u) / 2u : M;
        v[i] = r.d;
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->d_reps, v.data(), v.size() * sizeof(Replica), hipMemcpyHostToDevice));
    if (cells != h->ncell_total || doms != h->ndom_total || !h->d_cell2rep) {
        // flattened cell and domain indices -> replica (the geometry is fixed after build)
        std::vector<uint32_t> c2r(cells), d2r(doms);
        uint32_t maxcap = 0;
        for (size_t i = 0; i < h->reps.size(); ++i) {
            const HostReplica& r = h->reps[i];
            const uint32_t M = r.d.h * r.d.h * r.d.h;
            const uint32_t nd = h->p.pairing ? (M + 1u) / 2u : M;
            std::fill(c2r.begin() + r.d.cell_begin, c2r.begin() + r.d.cell_begin + r.ncells, (uint32_t)i);
            std::fill(d2r.begin() + r.d.dom_begin, d2r.begin() + r.d.dom_begin + nd, (uint32_t)i);
            maxcap = std::max(maxcap, r.cap);
        }
        dfree(h, h->d_cell2rep);
        dfree(h, h->d_dom2rep);
        dfree(h, h->d_lntab);
        dfree(h, h->d_plan_n);
        dfree(h, h->d_plan_heavy);
        dfree(h, h->d_plan_light);
        dfree(h, h->d_plan_geo_heavy);
        dfree(h, h->d_plan_geo_light);
        h->d_plan_geo_heavy = h->d_plan_geo_light = nullptr;
        h->d_cell2rep = h->d_dom2rep = nullptr;
        h->d_lntab = nullptr;
        h->d_plan_n = h->d_plan_heavy = h->d_plan_light = nullptr;
        // ln k for every count a domain can reach (two cells of capacity maxcap, plus one)
        h->lntab_n = (int32_t)(2u * maxcap + 2u);
        std::vector<double> lt((size_t)h->lntab_n, 0.0);
        for (int32_t k = 1; k < h->lntab_n; ++k) lt[(size_t)k] = std::log((double)k);
        HIP_TRY(h, dalloc(h, &h->d_cell2rep, c2r.size()));
        HIP_TRY(h, dalloc(h, &h->d_dom2rep, d2r.size()));
        HIP_TRY(h, dalloc(h, &h->d_lntab, lt.size()));
        HIP_TRY(h, dalloc(h, &h->d_plan_n, PLAN_N));
        HIP_TRY(h, dalloc(h, &h->d_plan_heavy, (size_t)8 * doms));
        HIP_TRY(h, dalloc(h, &h->d_plan_light, (size_t)8 * doms));
        HIP_TRY(h, dalloc(h, &h->d_plan_geo_heavy, (size_t)8 * doms));
        HIP_TRY(h, dalloc(h, &h->d_plan_geo_light, (size_t)8 * doms));
        HIP_TRY(h, hipMemset(h->d_plan_n, 0, PLAN_N * sizeof(uint32_t)));
        HIP_TRY(h, hipMemcpy(h->d_cell2rep, c2r.data(), c2r.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_dom2rep, d2r.data(), d2r.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_lntab, lt.data(), lt.size() * sizeof(double), hipMemcpyHostToDevice));
        h->ncell_total = cells;
        h->ndom_total = doms;
    }
    {
        // the shell thresholds of the learned proposal's features:
        // ceil((k rc / 16 / L 2^32)^2), k = 0..16, per replica
        std::vector<uint64_t> sh(17 * h->reps.size());
        for (size_t i = 0; i < h->reps.size(); ++i) {
            const HostReplica& r = h->reps[i];
            for (int k = 0; k <= 16; ++k) {
                const double t = (k * h->p.rc / 16.0 / r.L) * TWO32;
                sh[17 * i + k] = k ? (uint64_t)std::ceil(t * t) : 0;
            }
        }
        if (!h->d_R2sh) HIP_TRY(h, dalloc(h, &h->d_R2sh, sh.size()));
        HIP_TRY(h, hipMemcpy(h->d_R2sh, sh.data(), sh.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    }
    return CRMC_OK;
}

// He-uniform initial network: W1 and W2 from U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)),
// w3 from U(-sqrt(3 / 128), +sqrt(3 / 128)), biases zero; splitmix64 stream of seed
std::vector<float> initial_weights(uint64_t seed)
{
    std::vector<float> w(MLP_PARAMS, 0.0f);
    uint64_t x = seed;
    auto uniform = [&x]() {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0; // [-1, 1)
    };
    const double a1 = std::sqrt(6.0 / MLP_IN), a2 = std::sqrt(6.0 / MLP_H), a3 = std::sqrt(3.0 / MLP_H);
    for (int i = 0; i < MLP_B1; ++i) w[(size_t)i] = (float)(a1 * uniform());
    for (int i = MLP_W2; i < MLP_B2; ++i) w[(size_t)i] = (float)(a2 * uniform());
    for (int i = MLP_W3; i < MLP_B3; ++i) w[(size_t)i] = (float)(a3 * uniform());
    return w;
}

int ensure_params(crmc_t h)
{
    if (h->d_p32) return CRMC_OK;
    HIP_TRY(h, dalloc(h, &h->d_p32, MLP_PARAMS));
    HIP_TRY(h, dalloc(h, &h->d_p64, MLP_PARAMS));
    HIP_TRY(h, dalloc(h, &h->d_w1b, MLP_H * MLP_IN));
    HIP_TRY(h, dalloc(h, &h->d_w2b, MLP_H * MLP_H));
    HIP_TRY(h, dalloc(h, &h->d_adam_m, MLP_PARAMS));
    HIP_TRY(h, dalloc(h, &h->d_adam_v, MLP_PARAMS));
    HIP_TRY(h, dalloc(h, &h->d_grad, MLP_PARAMS));
    HIP_TRY(h, dalloc(h, &h->d_loss, 1));
    {
        const std::vector<float> w0 = initial_weights(h->p.seed ^ 0x5DEECE66Dull);
        HIP_TRY(h, hipMemcpy(h->d_p32, w0.data(), MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    }
    HIP_TRY(h, hipMemset(h->d_adam_m, 0, MLP_PARAMS * sizeof(float)));
    HIP_TRY(h, hipMemset(h->d_adam_v, 0, MLP_PARAMS * sizeof(float)));
    HIP_TRY(h, hipMemset(h->d_grad, 0, MLP_PARAMS * sizeof(float)));
    if (!h->learn_lds_set) {
        HIP_TRY(h, set_learn_lds_limit());
        h->learn_lds_set = true;
    }
    LearnArgs g{};
    g.p32 = h->d_p32;
    g.p64 = h->d_p64;
    g.w1b = h->d_w1b;
    g.w2b = h->d_w2b;
    HIP_TRY(h, launch_params_convert(g, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return CRMC_OK;
}

LearnArgs learn_args(crmc_t h)
{
    LearnArgs g;
    std::memset(&g, 0, sizeof g);
    // one workgroup per compute unit (the kernel holds the network in LDS)
    g.grid = (uint32_t)std::max(h->ncu, 1);
    g.R2sh = h->d_R2sh;
    g.p32 = h->d_p32;
    g.p64 = h->d_p64;
    g.w1b = h->d_w1b;
    g.w2b = h->d_w2b;
    g.data = h->collecting ? h->d_data : nullptr;
    g.data_n = h->d_data_n;
    g.data_cap = (uint64_t)h->data_cap;
    g.infer = h->learned ? 1 : 0;
    return g;
}

// The feature kernel's work items, per colour.  A colour's cells with sites
// number at most min(h^3, sites) per replica and hold ceil(count / 64) parts
// each, so min(h^3, sites) + ceil(sites / 64) items bound a replica's.
int ensure_learn_buffers(crmc_t h)
{
    uint64_t items = 0;
    for (auto& r : h->reps) {
        const uint64_t M = (uint64_t)r.d.h * r.d.h * r.d.h;
        items += std::min<uint64_t>(M, r.nsites) + (r.nsites + 63u) / 64u;
    }
    if (items * 8 > 0xFFFFFFFFull) return fail(h, CRMC_E_ARG, "too many sites for the learned proposal's work lists");
    if (items > h->lwork_cap || !h->d_lwork) {
        dfree(h, h->d_lwork);
        h->d_lwork = nullptr;
        const size_t m = (size_t)std::max<uint64_t>(items, 1);
        HIP_TRY(h, dalloc(h, &h->d_lwork, 8 * m));
        h->lwork_cap = (uint32_t)m;
    }
    if (!h->ncu) {
        int dev = 0;
        HIP_TRY(h, hipGetDevice(&dev));
        HIP_TRY(h, hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    return CRMC_OK;
}

hipError_t event_get(crmc_t h, hipEvent_t* e)
{
    if (!h->free_events.empty()) {
        *e = h->free_events.back();
        h->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// accumulate (and recycle) all but the newest `keep` timed launches
int drain_timing(crmc_t h, size_t keep)
{
    const size_t n = h->pending.size() > keep ? h->pending.size() - keep : 0;
    for (size_t i = 0; i < n; ++i) {
        auto& p = h->pending[i];
        HIP_TRY(h, hipEventSynchronize(p.b));
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, p.a, p.b));
        h->t_ms[p.kind] += ms;
        h->t_n[p.kind] += 1;
        h->free_events.push_back(p.a);
        h->free_events.push_back(p.b);
    }
    h->pending.erase(h->pending.begin(), h->pending.begin() + (ptrdiff_t)n);
    return CRMC_OK;
}

// enqueue one kernel, bracketed by events when timing is on
template <typename F>
int timed(crmc_t h, int kind, F&& launch)
{
    if (!h->timing) {
        HIP_TRY(h, launch());
        return CRMC_OK;
    }
    hipEvent_t a, b;
    HIP_TRY(h, event_get(h, &a));
    HIP_TRY(h, event_get(h, &b));
    HIP_TRY(h, hipEventRecord(a, h->stream));
    HIP_TRY(h, launch());
    HIP_TRY(h, hipEventRecord(b, h->stream));
    h->pending.push_back({kind, a, b});
    if (h->pending.size() > 4096) return drain_timing(h, 2048);
    return CRMC_OK;
}

constexpr int GRAPH_SWEEPS = 16;

// the start of a sweep: re-binning, then the plan of its eight phases
hipError_t enqueue_bin_plan(const SweepArgs& a, hipStream_t st)
{
    hipError_t e = launch_bin(a, st);
    return e == hipSuccess ? launch_plan(a, st) : e;
}

void drop_graphs(crmc_t h)
{
    for (auto& g : h->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// Sweeps as replays of captured graphs (GRAPH_SWEEPS at a time, then single
// sweeps) on the library's own stream, ordered after and before the caller's
// stream by events.  The kernels read the sweep counter and the conditions
// from device memory, so a captured graph stays valid across calls; it is
// recaptured when anything baked into its launch arguments changes.
int sweeps_by_graph(crmc_t h, const SweepArgs& a0, size_t lds, int64_t n, bool use_learn, const LearnArgs& lg)
{
    // A captured graph holds its kernels' arguments by value.  It is replayed
    // only while every argument (pointers, capacities, switches, launch
    // shape) is byte for byte the one it was captured with; anything else
    // (a buffer reallocated, even at the same address with another capacity)
    // recaptures.
    std::vector<uint8_t> key(sizeof(SweepArgs) + sizeof(LearnArgs) + sizeof(size_t) + 1, 0);
    std::memcpy(key.data(), &a0, sizeof(SweepArgs));
    if (use_learn) std::memcpy(key.data() + sizeof(SweepArgs), &lg, sizeof(LearnArgs));
    std::memcpy(key.data() + sizeof(SweepArgs) + sizeof(LearnArgs), &lds, sizeof(size_t));
    key.back() = use_learn ? 1 : 0;
    if (key != h->gargs) {
        drop_graphs(h);
        h->gargs.swap(key);
    }
    if (!h->gstream) HIP_TRY(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    if (!h->ev_in) HIP_TRY(h, hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    if (!h->ev_out) HIP_TRY(h, hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
    const int counts[2] = {1, GRAPH_SWEEPS};
    for (int g = 0; g < 2; ++g) {
        if (h->gexec[g]) continue;
        SweepArgs a = a0;
        HIP_TRY(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (int i = 0; i < counts[g] && err == hipSuccess; ++i) {
            err = enqueue_bin_plan(a, h->gstream);
            for (int col = 0; col < 8 && err == hipSuccess; ++col) {
                a.colour = col;
                if (use_learn) err = launch_learn(a, lg, h->gstream);
                if (err == hipSuccess) err = launch_phase(a, lds, h->gstream);
            }
            if (err == hipSuccess) err = launch_sweep_end(a, h->gstream);
        }
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(h->gstream, &graph);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(h, CRMC_E_DEVICE, std::string("graph capture failed: ") +
                                              hipGetErrorString(err != hipSuccess ? err : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&h->gexec[g], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            h->gexec[g] = nullptr;
            return fail(h, CRMC_E_DEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e3));
        }
    }
    HIP_TRY(h, hipEventRecord(h->ev_in, h->stream));
    HIP_TRY(h, hipStreamWaitEvent(h->gstream, h->ev_in, 0));
    for (; n >= GRAPH_SWEEPS; n -= GRAPH_SWEEPS) HIP_TRY(h, hipGraphLaunch(h->gexec[1], h->gstream));
    for (; n > 0; --n) HIP_TRY(h, hipGraphLaunch(h->gexec[0], h->gstream));
    HIP_TRY(h, hipEventRecord(h->ev_out, h->gstream));
    HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_out, 0));
    return CRMC_OK;
}

int check_device_errors(crmc_t h)
{
    uint32_t e = 0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(&e, h->d_err, sizeof e, hipMemcpyDeviceToHost));
    if (e & ERR_POOL) return fail(h, CRMC_E_DEVICE, "internal error: a domain did not fit its LDS pool");
    if (e & (ERR_BIN_CAPACITY | ERR_INSERT_CAPACITY))
        return fail(h, CRMC_E_CAPACITY, "a cell exceeded its record capacity (flags " + std::to_string(e) +
                                            "); rebuild with a larger cell_capacity");
    return CRMC_OK;
}

} // namespace

// ------------------------------------------------------------------------
// checkpoint and resume
// ------------------------------------------------------------------------
namespace {

constexpr char STATE_MAGIC[8] = {'C', 'R', 'M', 'C', 'S', 'T', 'A', 'T'};
constexpr uint32_t STATE_VERSION = 2;

struct Blob {
    std::vector<uint8_t> b;
    template <class T> void put(const T& v) { put_n(&v, 1); }
    template <class T> void put_n(const T* v, size_t n)
    {
        const uint8_t* p = reinterpret_cast<const uint8_t*>(v);
        b.insert(b.end(), p, p + n * sizeof(T));
    }
};

struct Cursor {
    const uint8_t* p;
    size_t n, at = 0;
    template <class T> bool get(T& v) { return get_n(&v, 1); }
    template <class T> bool get_n(T* v, size_t k)
    {
        const size_t bytes = k * sizeof(T);
        if (bytes > n - at) return false;
        std::memcpy(v, p + at, bytes);
        at += bytes;
        return true;
    }
};

// shape of a built replica that a state must match
struct RepShape {
    uint32_t n, cap, ncells, nsites, ngroups, ncores;
    double L;
};

RepShape shape_of(const HostReplica& r) { return RepShape{r.n, r.cap, r.ncells, r.nsites, r.ngroups, r.ncores, r.L}; }

// the capacity is storage only: a state fits any capacity that holds its cells
bool same_shape(const RepShape& a, const RepShape& b)
{
    return a.n == b.n && a.ncells == b.ncells && a.nsites == b.nsites && a.ngroups == b.ngroups &&
           a.ncores == b.ncores && a.L == b.L;
}

int serialize_state(crmc_t h, Blob& out)
{
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    int rc = check_device_errors(h);
    if (rc) return rc;
    out.put_n(STATE_MAGIC, 8);
    out.put(STATE_VERSION);
    out.put((uint32_t)h->reps.size());
    out.put((int32_t)h->p.precision);
    out.put((uint32_t)0);
    out.put(h->p.seed);
    out.put((int64_t)h->sweeps);
    out.put((uint64_t)h->md_steps);
    const int buf = (int)(h->sweeps & 1);
    for (const HostReplica& r : h->reps) {
        out.put(shape_of(r));
        out.put(r.E0);
        out.put(r.e0_kappa);
        uint32_t hiw = 0;
        HIP_TRY(h, hipMemcpy(&hiw, r.d.hiwater, sizeof hiw, hipMemcpyDeviceToHost));
        out.put(hiw);
        out.put((uint32_t)0);
        // records of every cell in list order (the order later picks depend on)
        std::vector<uint32_t> cnt(r.ncells);
        std::vector<uint4> rec((size_t)r.ncells * r.cap);
        HIP_TRY(h, hipMemcpy(cnt.data(), r.d.cnt[buf], r.ncells * sizeof(uint32_t), hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(rec.data(), r.d.rec[buf], rec.size() * sizeof(uint4), hipMemcpyDeviceToHost));
        out.put_n(cnt.data(), cnt.size());
        for (uint32_t c = 0; c < r.ncells; ++c) out.put_n(&rec[(size_t)c * r.cap], cnt[c]);
        std::vector<double> e(r.ncells);
        HIP_TRY(h, hipMemcpy(e.data(), r.d.e_acc, e.size() * sizeof(double), hipMemcpyDeviceToHost));
        out.put_n(e.data(), e.size());
        std::vector<uint64_t> occ(r.nsites);
        if (r.nsites) HIP_TRY(h, hipMemcpy(occ.data(), r.d.occupancy, occ.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
        out.put_n(occ.data(), occ.size());
        std::vector<int32_t> gc(2 * std::max<uint32_t>(r.ngroups, 1));
        HIP_TRY(h, hipMemcpy(gc.data(), r.d.group_count, gc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        out.put_n(gc.data(), gc.size());
        std::vector<int64_t> gh((size_t)r.hist_off[r.ngroups]);
        if (!gh.empty()) HIP_TRY(h, hipMemcpy(gh.data(), r.d.group_hist, gh.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        out.put_n(gh.data(), gh.size());
        int64_t tot[4];
        uint64_t mv[14];
        HIP_TRY(h, hipMemcpy(tot, r.d.totals, sizeof tot, hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(mv, r.d.moves, sizeof mv, hipMemcpyDeviceToHost));
        out.put_n(tot, 4);
        out.put_n(mv, 14);
        // the retained window of the series, oldest first
        const int64_t capn = r.d.series_cap;
        const int64_t first = std::max<int64_t>(0, h->sweeps - capn);
        std::vector<int32_t> all((size_t)capn * 4);
        HIP_TRY(h, hipMemcpy(all.data(), r.d.series, all.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        out.put(capn);
        for (int64_t s = first; s < h->sweeps; ++s) out.put_n(&all[(size_t)(s % capn) * 4], 4);
        out.put_n(r.d.lp_off, 2);
    }
    // proposal: switch, eps, and the network with its optimizer state when present
    out.put((uint32_t)h->learned);
    out.put(h->learn_eps);
    out.put((uint32_t)(h->d_p32 != nullptr));
    if (h->d_p32) {
        std::vector<float> w(MLP_PARAMS), m(MLP_PARAMS), v(MLP_PARAMS);
        HIP_TRY(h, hipMemcpy(w.data(), h->d_p32, MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(m.data(), h->d_adam_m, MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(v.data(), h->d_adam_v, MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
        out.put_n(w.data(), w.size());
        out.put_n(m.data(), m.size());
        out.put_n(v.data(), v.size());
        out.put(h->adam_t);
    }
    return CRMC_OK;
}

} // namespace

extern "C" {

double crmc_pIX_from_salt(double pIS, double pH, double pKw)
{
    const double pOH = pKw - pH;
    return -std::log10(std::pow(10.0, -pIS) + std::pow(10.0, -std::min(pH, pOH)));
}

int crmc_ungroup_fractions(double pH, double pKw, double pIS_pos, double pIS_neg, double pIX_pos, double pIX_neg,
                           double* out)
{
    if (!out || !std::isfinite(pH) || !std::isfinite(pKw) || !std::isfinite(pIS_pos) || !std::isfinite(pIS_neg) ||
        !std::isfinite(pIX_pos) || !std::isfinite(pIX_neg))
        return CRMC_E_ARG;
    // a subspecies' share of its combined ion is the ratio of their activities
    out[0] = std::pow(10.0, pIX_pos - pIS_pos);
    out[1] = std::pow(10.0, pIX_pos - pH);
    out[2] = std::pow(10.0, pIX_neg - pIS_neg);
    out[3] = std::pow(10.0, pIX_neg - (pKw - pH));
    return CRMC_OK;
}

const char* crmc_last_error(crmc_t h) { return h ? h->err.c_str() : "null handle"; }

int crmc_create(const crmc_params* p, crmc_t* out)
{
    if (!p || !out) return CRMC_E_ARG;
    *out = nullptr;
    if (p->n_replicas < 1 || p->n_replicas > (1 << 20)) return CRMC_E_ARG;
    if (p->precision != 32 && p->precision != 64) return CRMC_E_ARG;
    if (p->trials_per_cell < 1 || p->trials_per_cell > (1 << 20)) return CRMC_E_ARG;
    // the Coulomb cutoff must exceed the excluded-volume range 2^(1/6)
    if (!(p->rc > 1.2) || !(p->lB >= 0.0) || !(p->eps_wca >= 0.0) || !(p->rho0NA > 0.0)) return CRMC_E_ARG;
    if (p->lds_records < 0 || p->site_trials < 0 || p->site_trials > 4096) return CRMC_E_ARG;
    if (p->light_neighbours < 0 || p->light_neighbours > 65536) return CRMC_E_ARG;
    if (p->ion_trials < 0 || p->ion_trials > 4096 || (p->learned_proposal != 0 && p->learned_proposal != 1))
        return CRMC_E_ARG;
    if (p->learned_proposal && (!(p->learned_eps > 0.0) || p->learned_eps > 1.0)) return CRMC_E_ARG;
    if (p->workspace_bytes < 0 || (p->workspace && p->workspace_bytes < (int64_t)WS_ALIGN)) return CRMC_E_ARG;
    crmc_t h = new (std::nothrow) crmc_s;
    if (!h) return CRMC_E_NOMEM;
    h->p = *p;
    h->reps.resize((size_t)p->n_replicas);
    h->stream = (hipStream_t)p->stream;
    h->pool = p->lds_records > 0 ? p->lds_records : DEFAULT_POOL;
    h->learned = p->learned_proposal != 0;
    h->learn_eps = p->learned_proposal ? p->learned_eps : 0.1;
    crmc_cond c{};
    c.pH = 7.0; c.pKa = 4.5; c.pKb = p->pKb; c.pIX_pos = c.pIX_neg = 1.0; c.kappa = p->kappa;
    for (auto& r : h->reps) r.cond = c;
    if (p->workspace) h->ws.attach(p->workspace, (size_t)p->workspace_bytes);
    *out = h;
    return CRMC_OK;
}

int crmc_build_cells(crmc_t h, int32_t replica, double L, int32_t n_cells, int32_t cell_capacity, int32_t n,
                     const double* xyz, const int32_t* kind, const int32_t* charged, const int32_t* group,
                     int32_t n_cores, const double* core_xyz, const double* core_R)
{
    if (!h) return CRMC_E_ARG;
    if (replica < 0 || replica >= (int32_t)h->reps.size()) return fail(h, CRMC_E_ARG, "replica out of range");
    if (h->sweeps != 0) return fail(h, CRMC_E_STATE, "replicas must be built before the first sweep");
    if (!(L > 0.0) || n < 0 || (n > 0 && (!xyz || !kind)) || n_cores < 0 || (n_cores > 0 && (!core_xyz || !core_R)))
        return fail(h, CRMC_E_ARG, "invalid geometry arguments");
    if (n >= (int32_t)NO_SITE) return fail(h, CRMC_E_ARG, "too many particles in one replica");
    if (L < 4.0 * h->p.rc) return fail(h, CRMC_E_ARG, "box edge must be at least 4 rc");
    const uint64_t R2 = cutoff_R2(h->p.rc, L);
    uint32_t nc;
    if (n_cells == 0) {
        nc = (uint32_t)std::floor(L / h->p.rc);
        if (nc & 1u) --nc;
        while (nc >= 4 && !grid_ok(nc, R2)) nc -= 2;
        if (nc < 4) return fail(h, CRMC_E_ARG, "no valid cell grid");
    } else {
        if (n_cells < 4 || (n_cells & 1) || !grid_ok((uint32_t)n_cells, R2))
            return fail(h, CRMC_E_ARG, "n_cells must be even, >= 4 and give cells at least rc wide");
        nc = (uint32_t)n_cells;
    }
    if ((uint64_t)nc * nc * nc > (1ull << 31)) return fail(h, CRMC_E_ARG, "too many cells");
    for (int32_t i = 0; i < n; ++i) {
        const int k = kind[i];
        if (k < CRMC_ACID || k > CRMC_NEUTRAL) return fail(h, CRMC_E_ARG, "invalid particle kind");
        if (charged && (charged[i] != 0 && charged[i] != 1)) return fail(h, CRMC_E_ARG, "charged must be 0/1");
    }
    for (int32_t i = 0; i < n_cores; ++i)
        if (!(core_R[i] >= 0.5)) return fail(h, CRMC_E_ARG, "core radius must be >= 1/2");

    HostReplica& r = h->reps[(size_t)replica];
    if (r.built) free_replica(h, r);
    const uint32_t ncells = nc * nc * nc;

    // records in input order, then the stable binning into the unshifted grid
    std::vector<uint4> in((size_t)n);
    std::vector<std::vector<uint32_t>> lists(ncells);
    std::vector<uint32_t> site_cnt(ncells, 0);
    int64_t tot[4] = {0, 0, 0, 0};
    r.nA = r.nB = 0;
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t x = to_fixed(xyz[3 * i], L), y = to_fixed(xyz[3 * i + 1], L), z = to_fixed(xyz[3 * i + 2], L);
        const uint32_t k = (uint32_t)kind[i];
        const bool ion = k == KIND_XPOS || k == KIND_XNEG;
        const uint32_t ch = ion ? 1u : (charged ? (uint32_t)charged[i] : 0u);
        in[(size_t)i] = make_uint4(x, y, z, make_meta(k, ch, ion ? NO_SITE : (uint32_t)i));
        const uint32_t c = cell_of_h(x, nc) + nc * (cell_of_h(y, nc) + nc * cell_of_h(z, nc));
        lists[c].push_back((uint32_t)i);
        if (!ion) site_cnt[c]++;
        if (k == KIND_ACID) { r.nA++; tot[0] += ch; }
        if (k == KIND_BASE) { r.nB++; tot[1] += ch; }
        if (k == KIND_XPOS) tot[2]++;
        if (k == KIND_XNEG) tot[3]++;
    }
    uint32_t maxc = 0;
    for (uint32_t c = 0; c < ncells; ++c) maxc = std::max<uint32_t>(maxc, (uint32_t)lists[c].size());
    // Most sites any shifted cell can hold: on a grid four times finer, a
    // cell-wide interval touches at most five fine cells per dimension, so the
    // largest 5x5x5 block sum of fine-cell site counts bounds every shift.
    uint32_t site_bound = 0;
    {
        const uint32_t F = 4u * nc;
        std::vector<uint32_t> f((size_t)F * F * F, 0), g(f.size(), 0);
        for (int32_t i = 0; i < n; ++i) {
            const uint32_t k = (uint32_t)kind[i];
            if (k == KIND_XPOS || k == KIND_XNEG) continue;
            const uint4 v = in[(size_t)i];
            f[cell_of_h(v.x, F) + F * (cell_of_h(v.y, F) + (size_t)F * cell_of_h(v.z, F))]++;
        }
        for (int dim = 0; dim < 3; ++dim) {
            const size_t stride = dim == 0 ? 1 : (dim == 1 ? F : (size_t)F * F);
            for (size_t idx = 0; idx < f.size(); ++idx) {
                const size_t coord = (idx / stride) % F;
                uint32_t sum = 0;
                for (uint32_t o = 0; o < 5; ++o) {
                    const size_t cj = (coord + o) % F;
                    sum += f[idx + (cj - coord) * stride];
                }
                g[idx] = sum;
            }
            f.swap(g);
        }
        for (uint32_t v : f) site_bound = std::max(site_bound, v);
    }
    r.site_bound = site_bound;
    uint32_t cap;
    if (cell_capacity == 0) {
        // sites, as many counter-ions again, and room for salt
        cap = std::max<uint32_t>(64u, 2u * site_bound + 64u);
        cap = std::max<uint32_t>(cap, maxc + 32u);
        cap = (cap + 31u) & ~31u;
    } else {
        if (cell_capacity < 1 || (uint32_t)cell_capacity < maxc)
            return fail(h, CRMC_E_ARG, "cell_capacity below the particles already in one cell");
        cap = (uint32_t)cell_capacity;
    }

    // groups: dense indices in ascending order of the caller's ids
    std::map<int32_t, int32_t> gid;
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t k = (uint32_t)kind[i];
        if (k == KIND_XPOS || k == KIND_XNEG) continue;
        gid.emplace(group ? group[i] : 0, 0);
    }
    int32_t gi = 0;
    for (auto& kv : gid) kv.second = gi++;
    const uint32_t ngroups = (uint32_t)gid.size();
    std::vector<int32_t> site_group((size_t)std::max(n, 1), 0);
    std::vector<int32_t> gsize(ngroups, 0);
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t k = (uint32_t)kind[i];
        if (k == KIND_XPOS || k == KIND_XNEG) continue;
        const int32_t g = gid[group ? group[i] : 0];
        site_group[(size_t)i] = g;
        gsize[(size_t)g]++;
    }
    r.hist_off.assign(ngroups + 1, 0);
    for (uint32_t g = 0; g < ngroups; ++g) r.hist_off[g + 1] = r.hist_off[g] + gsize[g] + 1;

    // the initial state stays on the host until the device state is created
    r.init_rec.clear();
    r.init_rec.reserve((size_t)n);
    r.n_built = (int64_t)n;
    r.init_cnt.assign(ncells, 0u);
    for (uint32_t c = 0; c < ncells; ++c) {
        r.init_cnt[c] = (uint32_t)lists[c].size();
        for (uint32_t i : lists[c]) r.init_rec.push_back(in[i]);
    }
    r.init_cores.assign((size_t)std::max(n_cores, 1), make_uint4(0u, 0u, 0u, 0u));
    r.init_delta.assign((size_t)std::max(n_cores, 1), 0.0);
    for (int32_t i = 0; i < n_cores; ++i) {
        r.init_cores[(size_t)i] = make_uint4(to_fixed(core_xyz[3 * i], L), to_fixed(core_xyz[3 * i + 1], L),
                                             to_fixed(core_xyz[3 * i + 2], L), 0u);
        r.init_delta[(size_t)i] = core_R[i] - 0.5;
    }
    r.init_group = std::move(site_group);
    std::memcpy(r.init_tot, tot, sizeof tot);
    r.init_maxc = maxc;
    r.on_device = false;

    Replica& d = r.d;
    d = Replica{};
    const int64_t series_cap = DEFAULT_SERIES;
    d.series_cap = series_cap;
    // at least four cells per particle given: a cell's re-binning gathers a
    // few records at most, so one lane per cell keeps more cells in flight
    d.bin_sparse = (uint64_t)ncells >= 4ull * (uint64_t)std::max(n, 1) ? 1u : 0u;
    d.n = nc;
    d.h = nc / 2u;
    d.ncells = ncells;
    d.cap = cap;
    d.ncores = (uint32_t)n_cores;
    d.nsites = (uint32_t)n;
    d.ngroups = ngroups;
    d.key0 = (uint32_t)h->p.seed;
    d.key1 = (uint32_t)(h->p.seed >> 32) ^ (uint32_t)replica;
    d.L = L;
    d.scale = L / TWO32;
    d.lnZ0 = std::log(h->p.rho0NA) + 3.0 * std::log(L / TWO32);
    d.R2 = R2;
    r.L = L;
    r.n = nc;
    r.cap = cap;
    r.ncells = ncells;
    r.ncores = (uint32_t)n_cores;
    r.nsites = (uint32_t)n;
    r.ngroups = ngroups;
    set_conditions(h, r, r.cond);
    r.built = true;

    // the retained energy starts from scratch at the first sweep, once the
    // replica's screening length is known
    r.e0_kappa = std::nan("");
    return CRMC_OK;
}

// Device buffers of a built replica, in allocation order: (slot, bytes).
struct DevBuf {
    void** slot;
    size_t bytes;
};

static std::vector<DevBuf> replica_buffers(crmc_t h, HostReplica& r)
{
    Replica& d = r.d;
    const size_t ncells = r.ncells, nrec = ncells * r.cap, np = std::max<size_t>(r.nsites, 1);
    const size_t ng = std::max<uint32_t>(r.ngroups, 1), nh = (size_t)std::max(r.hist_off.empty() ? 0 : r.hist_off.back(), 1);
    const size_t nco = std::max<size_t>(r.ncores, 1);
    std::vector<DevBuf> v = {
        {(void**)&d.rec[0], nrec * sizeof(uint4)},   {(void**)&d.rec[1], nrec * sizeof(uint4)},
        {(void**)&d.cnt[0], ncells * 4},             {(void**)&d.cnt[1], ncells * 4},
        {(void**)&d.cnt0, ncells * 4},               {(void**)&d.e_acc, ncells * 8},
        {(void**)&d.occupancy, np * 8},              {(void**)&d.site_group, np * 4},
        {(void**)&d.group_count, 2 * ng * 4},        {(void**)&d.group_hist, nh * 8},
        {(void**)&d.group_hist_off, (r.ngroups + 1) * 4}, {(void**)&d.core_x, nco * sizeof(uint4)},
        {(void**)&d.core_delta, nco * 8},            {(void**)&d.totals, 4 * 8},
        {(void**)&d.moves, 14 * 8},                  {(void**)&d.series, (size_t)DEFAULT_SERIES * 4 * 4},
        {(void**)&d.ctr, (size_t)CTR_STRIPES * CTR_STRIDE * 4},
        {(void**)&d.phat, np * 8},                   {(void**)&d.nsc, ncells * 4},
        {(void**)&d.bnd, (r.n + 1) * 4},             {(void**)&d.lnW, r.n * 8},
        {(void**)&d.hiwater, 4},                     {(void**)&d.tab, sizeof(SweepTab)},
    };
    if (h->record_feat) v.push_back({(void**)&d.feat, np * MLP_IN * 4});
    return v;
}

// the device state of a replica from its initial state on the host
static int materialize_replica(crmc_t h, HostReplica& r)
{
    Replica& d = r.d;
    for (const DevBuf& b : replica_buffers(h, r)) {
        const hipError_t e = dalloc(h, (uint8_t**)b.slot, b.bytes);
        if (e != hipSuccess)
            return fail(h, e == hipErrorOutOfMemory ? CRMC_E_NOMEM : CRMC_E_DEVICE,
                        std::string(h->ws.base ? "workspace too small for the replicas' state (see "
                                                 "crmc_workspace_size): "
                                               : "device allocation failed: ") + hipGetErrorString(e));
    }
    const uint32_t ncells = r.ncells, cap = r.cap, nc = r.n, ngroups = r.ngroups;
    const size_t np = std::max<size_t>(r.nsites, 1);
    {
        // cell-major records, each cell's list padded to the capacity
        std::vector<uint4> cells((size_t)ncells * cap, make_uint4(0u, 0u, 0u, 0u));
        size_t k = 0;
        for (uint32_t c = 0; c < ncells; ++c)
            for (uint32_t j = 0; j < r.init_cnt[c]; ++j) cells[(size_t)c * cap + j] = r.init_rec[k++];
        HIP_TRY(h, hipMemcpy(d.rec[0], cells.data(), cells.size() * sizeof(uint4), hipMemcpyHostToDevice));
    }
    HIP_TRY(h, hipMemcpy(d.cnt[0], r.init_cnt.data(), ncells * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d.cnt[1], 0, ncells * sizeof(uint32_t)));
    HIP_TRY(h, hipMemset(d.e_acc, 0, ncells * sizeof(double)));
    HIP_TRY(h, hipMemset(d.occupancy, 0, np * sizeof(uint64_t)));
    HIP_TRY(h, hipMemset(d.phat, 0, np * sizeof(double)));
    if (d.feat) HIP_TRY(h, hipMemset(d.feat, 0, np * MLP_IN * sizeof(float)));
    HIP_TRY(h, hipMemset(d.nsc, 0, ncells * sizeof(uint32_t)));
    HIP_TRY(h, hipMemcpy(d.site_group, r.init_group.data(), r.init_group.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d.group_count, 0, 2 * std::max<uint32_t>(ngroups, 1) * sizeof(int32_t)));
    HIP_TRY(h, hipMemset(d.group_hist, 0, (size_t)std::max(r.hist_off[ngroups], 1) * sizeof(int64_t)));
    HIP_TRY(h, hipMemcpy(d.group_hist_off, r.hist_off.data(), (ngroups + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d.core_x, r.init_cores.data(), r.init_cores.size() * sizeof(uint4), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d.core_delta, r.init_delta.data(), r.init_delta.size() * sizeof(double),
                         hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d.totals, r.init_tot, sizeof r.init_tot, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d.moves, 0, 14 * sizeof(uint64_t)));
    HIP_TRY(h, hipMemset(d.ctr, 0, (size_t)CTR_STRIPES * CTR_STRIDE * sizeof(uint32_t)));
    HIP_TRY(h, hipMemset(d.series, 0, (size_t)d.series_cap * 4 * sizeof(int32_t)));
    {
        // cell boundaries b_k = ceil(k 2^32 / n) (b_n wraps to 0) and ln of the widths
        std::vector<uint32_t> b(nc + 1);
        std::vector<double> lw(nc);
        for (uint32_t k = 0; k <= nc; ++k) b[k] = (uint32_t)cell_lo_h(k, nc);
        for (uint32_t k = 0; k < nc; ++k) lw[k] = std::log((double)(cell_lo_h(k + 1, nc) - cell_lo_h(k, nc)));
        HIP_TRY(h, hipMemcpy(d.bnd, b.data(), b.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.lnW, lw.data(), lw.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.hiwater, &r.init_maxc, sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemset(d.tab, 0, sizeof(SweepTab)));
    }
    std::vector<uint4>().swap(r.init_rec);
    std::vector<uint32_t>().swap(r.init_cnt);
    std::vector<int32_t>().swap(r.init_group);
    r.on_device = true;
    return CRMC_OK;
}

// The handle's device state: the sweep counter, error flags and replica
// descriptors, then every built replica not yet on the device.
static int ready(crmc_t h)
{
    if (!h->d_sweep) {
        HIP_TRY(h, dalloc(h, &h->d_sweep, 1));
        HIP_TRY(h, dalloc(h, &h->d_err, 1));
        HIP_TRY(h, dalloc(h, &h->d_reps, h->reps.size()));
        HIP_TRY(h, hipMemset(h->d_sweep, 0, sizeof(uint64_t)));
        HIP_TRY(h, hipMemset(h->d_err, 0, sizeof(uint32_t)));
    }
    for (auto& r : h->reps)
        if (r.built && !r.on_device) {
            const int rc = materialize_replica(h, r);
            if (rc) return rc;
        }
    return CRMC_OK;
}

#define READY(h)                  \
    do {                          \
        const int rc_ = ready(h); \
        if (rc_) return rc_;      \
    } while (0)

// Bytes of device memory the handle's state needs at its current settings,
// each buffer rounded to the workspace granularity (the same buffers, in the
// same sizes, that ready(), upload_descriptors(), ensure_params(),
// ensure_learn_buffers() and state_energy() allocate).
static size_t state_bytes(crmc_t h)
{
    size_t b = WS_ALIGN; // slack for a workspace pointer that is not 256-byte aligned
    auto add = [&b](size_t x) { b += ws_round(x); };
    add(sizeof(uint64_t));
    add(sizeof(uint32_t));
    add(sizeof(Replica) * h->reps.size());
    uint64_t cells = 0, doms = 0, items = 0;
    uint32_t maxcap = 0;
    size_t max_cells = 1;
    for (auto& r : h->reps) {
        if (!r.built) continue;
        for (const DevBuf& bf : replica_buffers(h, r)) add(bf.bytes);
        const uint64_t M = (uint64_t)r.d.h * r.d.h * r.d.h;
        cells += r.ncells;
        doms += h->p.pairing ? (M + 1u) / 2u : M;
        items += std::min<uint64_t>(M, r.nsites) + (r.nsites + 63u) / 64u;
        maxcap = std::max(maxcap, r.cap);
        max_cells = std::max<size_t>(max_cells, r.ncells);
    }
    // flattened indices, the ln k table, the plan, the feature shells
    add(cells * 4);
    add(doms * 4);
    add((2 * (size_t)maxcap + 2) * 8);
    add(PLAN_N * 4);
    add(8 * doms * 4);
    add(8 * doms * 4);
    add(8 * doms * sizeof(uint4));
    add(8 * doms * sizeof(uint4));
    add(17 * h->reps.size() * 8);
    // the network (FP32 masters, FP64 and BF16 copies), Adam, the gradient,
    // the learned proposal's work items and the training-row counter
    add(MLP_PARAMS * 4);
    add(MLP_PARAMS * 8);
    add(MLP_H * MLP_IN * 2);
    add(MLP_H * MLP_H * 2);
    for (int i = 0; i < 3; ++i) add(MLP_PARAMS * 4);
    add(8);
    add(8 * std::max<uint64_t>(items, 1) * sizeof(LearnItem));
    add(8);
    // the from-scratch energy's per-cell sums
    add(sizeof(Replica));
    add(max_cells * 8);
    return b;
}

static int state_energy(crmc_t h, HostReplica& r, double* out)
{
    Replica* d_one = nullptr;
    double* d_e = nullptr;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, dalloc(h, &d_one, 1));
    HIP_TRY(h, dalloc(h, &d_e, r.ncells));
    HIP_TRY(h, hipMemcpy(d_one, &r.d, sizeof(Replica), hipMemcpyHostToDevice));
    HIP_TRY(h, launch_energy(d_one, r.d, h->p.lB, h->p.eps_wca, h->p.ion_coupling, (int)(h->sweeps & 1), d_e,
                             h->stream));
    std::vector<double> pe(r.ncells);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(pe.data(), d_e, r.ncells * sizeof(double), hipMemcpyDeviceToHost));
    dfree(h, d_one);
    dfree(h, d_e);
    double E = 0.0;
    for (double v : pe) E += v;
    *out = E;
    return CRMC_OK;
}

int crmc_workspace_size(crmc_t h, int64_t* bytes)
{
    if (!h || !bytes) return fail(h, CRMC_E_ARG, "bad arguments");
    for (const HostReplica& r : h->reps)
        if (!r.built) return fail(h, CRMC_E_STATE, "build every replica before sizing the workspace");
    *bytes = (int64_t)state_bytes(h);
    return CRMC_OK;
}

int crmc_set_workspace(crmc_t h, void* workspace, int64_t bytes)
{
    if (!h || !workspace || bytes < (int64_t)WS_ALIGN) return fail(h, CRMC_E_ARG, "bad workspace");
    if (h->device_state || h->ws.base)
        return fail(h, CRMC_E_STATE, "the handle already has device memory; attach the workspace right after "
                                     "creating and building");
    h->ws.attach(workspace, (size_t)bytes);
    return CRMC_OK;
}

int crmc_memory(crmc_t h, int64_t* own_bytes, int64_t* workspace_used, int64_t* workspace_largest_free)
{
    if (!h) return CRMC_E_ARG;
    int64_t own = 0;
    for (const auto& kv : h->own) own += (int64_t)kv.second;
    if (own_bytes) *own_bytes = own;
    if (workspace_used) *workspace_used = (int64_t)h->ws.used;
    if (workspace_largest_free) *workspace_largest_free = (int64_t)h->ws.largest_free();
    return CRMC_OK;
}

int crmc_sweep_ex(crmc_t h, const crmc_cond* per_replica, int64_t n_sweeps)
{
    if (!h || !per_replica || n_sweeps < 0) return fail(h, CRMC_E_ARG, "invalid sweep arguments");
    uint32_t maxcap = 0;
    for (auto& r : h->reps) {
        if (!r.built) return fail(h, CRMC_E_STATE, "every replica must be built before sweeping");
        maxcap = std::max(maxcap, r.cap);
    }
    READY(h);
    if ((uint64_t)h->sweeps + (uint64_t)n_sweeps >= (1ull << 32))
        return fail(h, CRMC_E_ARG, "sweep counter would exceed 2^32");
    for (size_t i = 0; i < h->reps.size(); ++i) {
        const crmc_cond& c = per_replica[i];
        if (!std::isfinite(c.pH) || !std::isfinite(c.pKa) || !std::isfinite(c.pKb) || !std::isfinite(c.pIX_pos) ||
            !std::isfinite(c.pIX_neg) || !(c.kappa >= 0.0))
            return fail(h, CRMC_E_ARG, "invalid conditions");
        set_conditions(h, h->reps[i], c);
    }
    // The energy function depends on kappa: where it changed (or before the
    // first sweep) the retained energy restarts from a from-scratch sum.
    for (auto& r : h->reps) {
        if (r.e0_kappa == r.d.kappa) continue;
        double E = 0.0;
        int rc = state_energy(h, r, &E);
        if (rc) return rc;
        HIP_TRY(h, hipMemset(r.d.e_acc, 0, r.ncells * sizeof(double)));
        r.E0 = E;
        r.e0_kappa = r.d.kappa;
    }
    // the pool of a heavy domain must hold both cells' lists (2 cap), the ln k
    // table (2 cap + 2 doubles), up to 64 cores with their Deltas (96 records)
    // and, with the learned proposal, a double per list slot (cap records)
    const int pool_floor = (int)((h->learned ? 4 : 3) * maxcap + 128);
    if (h->pool < pool_floor) h->pool = pool_floor;
    h->pool = (h->pool + 3) & ~3; // four equal quarters for light domains
    const size_t lds = (size_t)h->pool * sizeof(uint4);
    int dev = 0, maxlds = 0;
    HIP_TRY(h, hipGetDevice(&dev));
    HIP_TRY(h, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds + 1024 > (size_t)maxlds)
        return fail(h, CRMC_E_ARG, "cell capacity too large for on-chip staging (" + std::to_string(lds) +
                                        " bytes of LDS needed)");
    if (lds > h->lds_attr) {
        HIP_TRY(h, set_phase_lds_limit(lds));
        h->lds_attr = lds;
    }
    const bool use_learn = h->learned || h->collecting;
    int rc = CRMC_OK;
    if (use_learn) {
        rc = ensure_params(h);
        if (!rc) rc = ensure_learn_buffers(h);
        if (rc) return rc;
    }
    rc = upload_descriptors(h);
    if (rc) return rc;
    SweepArgs a = base_args(h);
    LearnArgs lg{};
    if (use_learn) {
        a.lwork = h->d_lwork;
        a.lwork_cap = h->lwork_cap;
        lg = learn_args(h);
    }
    if (h->p.use_graph && !h->timing) {
        rc = sweeps_by_graph(h, a, lds, n_sweeps, use_learn, lg);
        if (rc) return rc;
        h->sweeps += n_sweeps;
        return CRMC_OK;
    }
    hipStream_t st = h->stream;
    for (int64_t i = 0; i < n_sweeps; ++i) {
        rc = timed(h, 0, [&] { return enqueue_bin_plan(a, st); });
        if (rc) return rc;
        for (int col = 0; col < 8; ++col) {
            a.colour = col;
            if (use_learn) {
                rc = timed(h, 0, [&] { return launch_learn(a, lg, st); });
                if (rc) return rc;
            }
            rc = timed(h, 1, [&] { return launch_phase(a, lds, st); });
            if (rc) return rc;
        }
        rc = timed(h, 2, [&] { return launch_sweep_end(a, st); });
        if (rc) return rc;
        h->sweeps++;
    }
    return CRMC_OK;
}

// A larger record capacity per cell for a replica on the device: both record
// buffers re-laid out with the new stride (the current one keeps its lists;
// the other is rewritten by the next re-binning).  The flattened tables (the
// ln k table reaches twice the capacity) are rebuilt by the next sweep.
static int grow_capacity(crmc_t h, HostReplica& r, uint32_t new_cap)
{
    if (new_cap <= r.cap) return CRMC_OK;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const size_t nrec = (size_t)r.ncells * new_cap;
    for (int b = 0; b < 2; ++b) {
        uint4* fresh = nullptr;
        HIP_TRY(h, dalloc(h, &fresh, nrec));
        HIP_TRY(h, hipMemcpy2D(fresh, new_cap * sizeof(uint4), r.d.rec[b], r.cap * sizeof(uint4),
                               r.cap * sizeof(uint4), r.ncells, hipMemcpyDeviceToDevice));
        dfree(h, r.d.rec[b]);
        r.d.rec[b] = fresh;
    }
    r.cap = new_cap;
    r.d.cap = new_cap;
    for (double*& q : r.md_vel) { dfree(h, q); q = nullptr; }
    dfree(h, r.md_force);
    r.md_force = nullptr;
    h->ncell_total = 0; // rebuild the flattened tables and the ln k table
    drop_graphs(h);
    return CRMC_OK;
}

int crmc_sweep_recover(crmc_t h, const crmc_cond* per_replica, int64_t n_sweeps, int64_t chunk,
                       int32_t* recoveries)
{
    if (!h || !per_replica || n_sweeps < 0 || chunk < 1) return fail(h, CRMC_E_ARG, "invalid arguments");
    for (auto& r : h->reps)
        if (!r.built) return fail(h, CRMC_E_STATE, "every replica must be built before sweeping");
    READY(h);
    int32_t nrec = 0;
    int rc = check_device_errors(h);
    if (rc) return rc;
    Blob good;
    rc = serialize_state(h, good);
    if (rc) return rc;
    for (int64_t done = 0; done < n_sweeps;) {
        const int64_t k = std::min(chunk, n_sweeps - done);
        rc = crmc_sweep_ex(h, per_replica, k);
        if (!rc) rc = check_device_errors(h);
        if (rc == CRMC_E_CAPACITY) {
            // roll back to the last good state with more room in every cell,
            // then replay the same sweeps (the random numbers are counter based)
            if (++nrec > 16) return fail(h, CRMC_E_CAPACITY, "cell capacity still exceeded after 16 enlargements");
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            HIP_TRY(h, hipMemset(h->d_err, 0, sizeof(uint32_t)));
            for (auto& r : h->reps) {
                const uint32_t grown = ((r.cap + std::max<uint32_t>(32u, r.cap / 2u)) + 31u) & ~31u;
                rc = grow_capacity(h, r, grown);
                if (rc) return rc;
            }
            rc = crmc_import_state(h, good.b.data(), (int64_t)good.b.size());
            if (rc) return rc;
            continue;
        }
        if (rc) return rc;
        done += k;
        if (done < n_sweeps) {
            good.b.clear();
            rc = serialize_state(h, good);
            if (rc) return rc;
        }
    }
    if (recoveries) *recoveries = nrec;
    return CRMC_OK;
}

int crmc_md(crmc_t h, int64_t n_steps, double dt, double gamma)
{
    if (!h || n_steps < 0 || !(dt > 0.0) || !(gamma >= 0.0) || !std::isfinite(dt) || !std::isfinite(gamma))
        return fail(h, CRMC_E_ARG, "invalid molecular-dynamics arguments");
    uint32_t maxcap = 0;
    for (auto& r : h->reps) {
        if (!r.built) return fail(h, CRMC_E_STATE, "every replica must be built before molecular dynamics");
        maxcap = std::max(maxcap, r.cap);
    }
    READY(h);
    int rc = upload_descriptors(h);
    if (rc) return rc;
    if (n_steps == 0) return CRMC_OK;
    // per-slot velocities (both record buffers) and forces, made at the first block
    std::vector<double*> vel(2 * h->reps.size()), frc(h->reps.size());
    for (size_t i = 0; i < h->reps.size(); ++i) {
        HostReplica& r = h->reps[i];
        const size_t m = (size_t)r.ncells * r.cap * 3;
        for (int b = 0; b < 2; ++b)
            if (!r.md_vel[b]) HIP_TRY(h, dalloc(h, &r.md_vel[b], m));
        if (!r.md_force) HIP_TRY(h, dalloc(h, &r.md_force, m));
        vel[2 * i] = r.md_vel[0];
        vel[2 * i + 1] = r.md_vel[1];
        frc[i] = r.md_force;
    }
    if (!h->d_md_vel) HIP_TRY(h, dalloc(h, &h->d_md_vel, vel.size()));
    if (!h->d_md_force) HIP_TRY(h, dalloc(h, &h->d_md_force, frc.size()));
    HIP_TRY(h, hipMemcpy(h->d_md_vel, vel.data(), vel.size() * sizeof(double*), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_md_force, frc.data(), frc.size() * sizeof(double*), hipMemcpyHostToDevice));
    MdArgs m;
    std::memset(&m, 0, sizeof m);
    m.reps = h->d_reps;
    m.cell2rep = h->d_cell2rep;
    m.ncell_total = h->ncell_total;
    m.vel = h->d_md_vel;
    m.force = h->d_md_force;
    m.err = h->d_err;
    m.lB = h->p.lB;
    m.eps = h->p.eps_wca;
    m.dt = dt;
    m.gamma = gamma;
    m.noise = std::sqrt(2.0 * gamma / dt);
    m.ion_coupling = h->p.ion_coupling;
    m.precision = h->p.precision;
    const int buf0 = (int)(h->sweeps & 1);
    int buf = buf0;
    HIP_TRY(h, launch_md_block(m, buf0, h->md_steps, n_steps, maxcap, h->stream, &buf));
    if (buf != buf0) {
        // the sweeps read the records of buffer (sweeps & 1)
        for (auto& r : h->reps) {
            HIP_TRY(h, hipMemcpyAsync(r.d.rec[buf0], r.d.rec[buf], (size_t)r.ncells * r.cap * sizeof(uint4),
                                      hipMemcpyDeviceToDevice, h->stream));
            HIP_TRY(h, hipMemcpyAsync(r.d.cnt[buf0], r.d.cnt[buf], (size_t)r.ncells * sizeof(uint32_t),
                                      hipMemcpyDeviceToDevice, h->stream));
        }
    }
    h->md_steps += (uint64_t)n_steps;
    rc = check_device_errors(h);
    if (rc) return rc;
    // positions moved: the retained energy restarts from a from-scratch sum
    for (auto& r : h->reps) {
        double E = 0.0;
        rc = state_energy(h, r, &E);
        if (rc) return rc;
        HIP_TRY(h, hipMemset(r.d.e_acc, 0, r.ncells * sizeof(double)));
        r.E0 = E;
        r.e0_kappa = r.d.kappa;
    }
    return CRMC_OK;
}

// Launch shapes chosen by crmc_autotune in this process, keyed by the device,
// precision, schedule, proposal, seed and the replicas' grids, capacities,
// cores and sizes: a handle rebuilt on the same inputs tunes once.
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<int, int>> g_tune_cache;

static std::string tune_key(crmc_t h, int dev)
{
    std::string k;
    char b[160];
    std::snprintf(b, sizeof b, "d%d p%d t%d s%d i%d q%d f%d l%d k%llu;", dev, h->p.precision, h->p.trials_per_cell,
                  h->p.site_trials, h->p.ion_trials, h->p.pairing, h->p.fixed_grid, (int)h->learned,
                  (unsigned long long)h->p.seed);
    k += b;
    for (auto& r : h->reps) {
        std::snprintf(b, sizeof b, "%u,%u,%u,%u,%lld;", r.n, r.cap, r.ncores, r.nsites, (long long)r.n_built);
        k += b;
    }
    return k;
}

int crmc_autotune(crmc_t h, const crmc_cond* per_replica, int32_t sweeps_per_candidate, crmc_tune* out)
{
    if (!h || !per_replica || !out || sweeps_per_candidate < 1 || sweeps_per_candidate > 100000)
        return fail(h, CRMC_E_ARG, "invalid autotune arguments");
    uint32_t maxcap = 0;
    for (auto& r : h->reps) {
        if (!r.built) return fail(h, CRMC_E_STATE, "every replica must be built before tuning");
        maxcap = std::max(maxcap, r.cap);
    }
    int dev = 0, maxlds = 0;
    HIP_TRY(h, hipGetDevice(&dev));
    HIP_TRY(h, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const std::string key = tune_key(h, dev);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            // the same configuration was tuned before in this process
            std::memset(out, 0, sizeof *out);
            h->p.light_neighbours = it->second.first;
            h->pool = it->second.second;
            out->light_neighbours = it->second.first;
            out->lds_records = it->second.second;
            out->reserved = 1;
            return CRMC_OK;
        }
    }
    const int pool_min = (int)((h->learned ? 4 : 3) * maxcap + 128);
    const int pool_max = (maxlds - 1024) / (int)sizeof(uint4);
    const int light_c[] = {256, 512, 768, 1024, 1536};
    const int pool_c[] = {pool_min, 3072, 4096, 6144, 8192};
    std::memset(out, 0, sizeof *out);
    const int keep_light = h->p.light_neighbours, keep_pool = h->pool;
    const bool keep_timing = h->timing;
    h->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    double best = 1e300;
    int best_l = keep_light, best_p = keep_pool, rc = CRMC_OK;
    for (int pc : pool_c) {
        if (pc < pool_min || pc > pool_max) continue;
        bool dup = false;
        for (int i = 0; i < out->n_candidates; ++i) dup = dup || out->cand_lds[i] == ((pc + 3) & ~3);
        if (dup) continue;
        for (int lc : light_c) {
            if (out->n_candidates >= CRMC_TUNE_MAX) break;
            h->p.light_neighbours = lc;
            h->pool = pc;
            rc = crmc_sweep_ex(h, per_replica, 1); // warm-up: capture, LDS limit
            if (rc) break;
            if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = CRMC_E_DEVICE; break; }
            rc = crmc_sweep_ex(h, per_replica, sweeps_per_candidate);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = CRMC_E_DEVICE;
                break;
            }
            const int i = out->n_candidates++;
            out->cand_light[i] = lc;
            out->cand_lds[i] = h->pool;
            out->ms_per_sweep[i] = ms / sweeps_per_candidate;
            if (out->ms_per_sweep[i] < best) {
                best = out->ms_per_sweep[i];
                best_l = lc;
                best_p = h->pool;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->timing = keep_timing;
    if (rc) {
        h->p.light_neighbours = keep_light;
        h->pool = keep_pool;
        return rc;
    }
    h->p.light_neighbours = best_l;
    h->pool = best_p;
    out->light_neighbours = best_l;
    out->lds_records = best_p;
    out->best_ms_per_sweep = best;
    out->sweeps_used = (int64_t)out->n_candidates * (sweeps_per_candidate + 1);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = std::make_pair(best_l, best_p);
    }
    return CRMC_OK;
}

int crmc_set_proposal(crmc_t h, int32_t learned, double eps)
{
    if (!h || (learned != 0 && learned != 1)) return fail(h, CRMC_E_ARG, "invalid proposal");
    if (learned && (!(eps > 0.0) || eps > 1.0)) return fail(h, CRMC_E_ARG, "eps must lie in (0, 1]");
    h->learned = learned != 0;
    if (learned) h->learn_eps = eps;
    return CRMC_OK;
}

int crmc_set_proposal_weights(crmc_t h, const float* w, int64_t n)
{
    if (!h || !w || n != MLP_PARAMS) return fail(h, CRMC_E_ARG, "expected the network's parameters");
    int rc = ensure_params(h);
    if (rc) return rc;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->d_p32, w, MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    LearnArgs g = learn_args(h);
    HIP_TRY(h, launch_params_convert(g, h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_adam_m, 0, MLP_PARAMS * sizeof(float), h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_adam_v, 0, MLP_PARAMS * sizeof(float), h->stream));
    h->adam_t = 0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return CRMC_OK;
}

int crmc_set_proposal_offsets(crmc_t h, int32_t replica, double acid, double base)
{
    if (!h || replica < 0 || replica >= (int32_t)h->reps.size() || !std::isfinite(acid) || !std::isfinite(base))
        return fail(h, CRMC_E_ARG, "invalid replica or offset");
    h->reps[(size_t)replica].d.lp_off[0] = acid;
    h->reps[(size_t)replica].d.lp_off[1] = base;
    return CRMC_OK;
}

int crmc_get_site_probabilities(crmc_t h, int32_t replica, double* out, int64_t n)
{
    if (!h || !out || replica < 0 || replica >= (int32_t)h->reps.size())
        return fail(h, CRMC_E_ARG, "invalid replica or buffer");
    const HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    if (n < (int64_t)r.nsites) return fail(h, CRMC_E_ARG, "buffer smaller than the replica's particle count");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(out, r.d.phat, (size_t)r.nsites * sizeof(double), hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_init_proposal_weights(crmc_t h, uint64_t seed)
{
    if (!h) return CRMC_E_ARG;
    const std::vector<float> w = initial_weights(seed);
    return crmc_set_proposal_weights(h, w.data(), MLP_PARAMS);
}

int crmc_get_proposal_weights(crmc_t h, float* w, int64_t n)
{
    if (!h || !w || n != MLP_PARAMS) return fail(h, CRMC_E_ARG, "expected room for the network's parameters");
    int rc = ensure_params(h);
    if (rc) return rc;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(w, h->d_p32, MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_collect_training(crmc_t h, int64_t capacity)
{
    if (!h || capacity < 0 || capacity > (int64_t)1 << 28) return fail(h, CRMC_E_ARG, "invalid capacity");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    dfree(h, h->d_data);
    h->d_data = nullptr;
    h->data_cap = 0;
    h->collecting = false;
    if (!h->d_data_n) HIP_TRY(h, dalloc(h, &h->d_data_n, 1));
    HIP_TRY(h, hipMemset(h->d_data_n, 0, sizeof(unsigned long long)));
    if (capacity == 0) return CRMC_OK;
    HIP_TRY(h, dalloc(h, &h->d_data, (size_t)capacity * (MLP_IN + 1)));
    h->data_cap = capacity;
    h->collecting = true;
    return CRMC_OK;
}

int crmc_training_rows(crmc_t h, int64_t* n)
{
    if (!h || !n) return CRMC_E_ARG;
    *n = 0;
    if (!h->d_data_n) return CRMC_OK;
    unsigned long long v = 0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(&v, h->d_data_n, sizeof v, hipMemcpyDeviceToHost));
    *n = (int64_t)std::min<unsigned long long>(v, (unsigned long long)h->data_cap);
    return CRMC_OK;
}

int crmc_read_training(crmc_t h, int64_t first, int64_t count, float* out)
{
    int64_t n = 0;
    int rc = crmc_training_rows(h, &n);
    if (rc) return rc;
    if (!out || first < 0 || count < 0 || first + count > n) return fail(h, CRMC_E_ARG, "rows out of range");
    HIP_TRY(h, hipMemcpy(out, h->d_data + (size_t)first * (MLP_IN + 1), (size_t)count * (MLP_IN + 1) * sizeof(float),
                         hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_load_training(crmc_t h, const float* rows, int64_t n)
{
    if (!h || n < 0 || n > (int64_t)1 << 28 || (n > 0 && !rows)) return fail(h, CRMC_E_ARG, "invalid rows");
    int rc = crmc_collect_training(h, 0);
    if (rc) return rc;
    if (n == 0) return CRMC_OK;
    HIP_TRY(h, dalloc(h, &h->d_data, (size_t)n * (MLP_IN + 1)));
    h->data_cap = n;
    HIP_TRY(h, hipMemcpy(h->d_data, rows, (size_t)n * (MLP_IN + 1) * sizeof(float), hipMemcpyHostToDevice));
    const unsigned long long nn = (unsigned long long)n;
    HIP_TRY(h, hipMemcpy(h->d_data_n, &nn, sizeof nn, hipMemcpyHostToDevice));
    return CRMC_OK;
}

int crmc_record_features(crmc_t h, int32_t on)
{
    if (!h || (on != 0 && on != 1)) return fail(h, CRMC_E_ARG, "invalid switch");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (auto& r : h->reps) {
        dfree(h, r.d.feat);
        r.d.feat = nullptr;
        if (!on || !r.built) continue;
        const size_t m = (size_t)std::max<uint32_t>(r.nsites, 1) * MLP_IN;
        HIP_TRY(h, dalloc(h, &r.d.feat, m));
        HIP_TRY(h, hipMemset(r.d.feat, 0, m * sizeof(float)));
    }
    h->record_feat = on != 0;
    return CRMC_OK;
}

int crmc_get_site_features(crmc_t h, int32_t replica, float* out, int64_t n)
{
    if (!h || !out || replica < 0 || replica >= (int32_t)h->reps.size())
        return fail(h, CRMC_E_ARG, "invalid replica or buffer");
    const HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    if (!r.d.feat) return fail(h, CRMC_E_STATE, "feature recording is off");
    if (n < (int64_t)r.nsites * MLP_IN) return fail(h, CRMC_E_ARG, "buffer smaller than 32 values per particle");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(out, r.d.feat, (size_t)r.nsites * MLP_IN * sizeof(float), hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_train(crmc_t h, int32_t epochs, int32_t batch, double lr, uint64_t seed, double* last_loss)
{
    if (!h || epochs < 0 || batch < 16 || batch > 65536 || !(lr > 0.0)) return fail(h, CRMC_E_ARG, "invalid training");
    int64_t n = 0;
    int rc = crmc_training_rows(h, &n);
    if (rc) return rc;
    if (n < batch) return fail(h, CRMC_E_STATE, "fewer training rows than one batch");
    rc = ensure_params(h);
    if (rc) return rc;
    LearnArgs g = learn_args(h);
    int* d_rows = nullptr;
    HIP_TRY(h, dalloc(h, &d_rows, (size_t)n));
    std::vector<int> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (int)i;
    uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
    double epoch_loss = 0.0;
    const int64_t nb = n / batch;
    for (int e = 0; e < epochs; ++e) {
        for (int64_t i = n - 1; i > 0; --i) { // Fisher-Yates with a 64-bit LCG
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            const int64_t j = (int64_t)((st >> 33) % (uint64_t)(i + 1));
            std::swap(perm[(size_t)i], perm[(size_t)j]);
        }
        if (hipMemcpy(d_rows, perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            dfree(h, d_rows);
            return fail(h, CRMC_E_DEVICE, "row upload failed");
        }
        hipError_t err = hipMemsetAsync(h->d_loss, 0, sizeof(double), h->stream);
        for (int64_t b = 0; b < nb && err == hipSuccess; ++b) {
            err = launch_mlp_grad(g, h->d_data, d_rows + b * batch, batch, 1.0f / batch, h->d_grad, h->d_loss,
                                  h->stream);
            ++h->adam_t;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)h->adam_t));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)h->adam_t));
            if (err == hipSuccess) err = launch_adam(g, h->d_grad, h->d_adam_m, h->d_adam_v, (float)lr, c1, c2, h->stream);
        }
        double lsum = 0.0;
        if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
        if (err == hipSuccess) err = hipMemcpy(&lsum, h->d_loss, sizeof(double), hipMemcpyDeviceToHost);
        if (err != hipSuccess) {
            dfree(h, d_rows);
            return fail(h, CRMC_E_DEVICE, std::string("training failed: ") + hipGetErrorString(err));
        }
        epoch_loss = lsum / (double)nb;
    }
    dfree(h, d_rows);
    if (last_loss) *last_loss = epoch_loss;
    return CRMC_OK;
}

int crmc_mlp_forward(crmc_t h, const float* X, int32_t n, float* logits)
{
    if (!h || !X || !logits || n < 0) return fail(h, CRMC_E_ARG, "invalid arguments");
    int rc = ensure_params(h);
    if (rc) return rc;
    float *dX = nullptr, *dz = nullptr;
    HIP_TRY(h, dalloc(h, &dX, (size_t)n * MLP_IN));
    HIP_TRY(h, dalloc(h, &dz, (size_t)n));
    hipError_t e = hipMemcpy(dX, X, (size_t)n * MLP_IN * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_fwd(learn_args(h), dX, n, dz, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(logits, dz, (size_t)n * sizeof(float), hipMemcpyDeviceToHost);
    dfree(h, dX);
    dfree(h, dz);
    if (e != hipSuccess) return fail(h, CRMC_E_DEVICE, hipGetErrorString(e));
    return CRMC_OK;
}

int crmc_mlp_gradient(crmc_t h, const float* rows, int32_t n, float* grad, double* loss)
{
    if (!h || !rows || !grad || n < 1) return fail(h, CRMC_E_ARG, "invalid arguments");
    int rc = ensure_params(h);
    if (rc) return rc;
    float* dD = nullptr;
    int* dr = nullptr;
    HIP_TRY(h, dalloc(h, &dD, (size_t)n * (MLP_IN + 1)));
    HIP_TRY(h, dalloc(h, &dr, (size_t)n));
    std::vector<int> idx((size_t)n);
    for (int i = 0; i < n; ++i) idx[(size_t)i] = i;
    hipError_t e = hipMemcpy(dD, rows, (size_t)n * (MLP_IN + 1) * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dr, idx.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_grad, 0, MLP_PARAMS * sizeof(float), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_loss, 0, sizeof(double), h->stream);
    if (e == hipSuccess) e = launch_mlp_grad(learn_args(h), dD, dr, n, 1.0f / n, h->d_grad, h->d_loss, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(grad, h->d_grad, MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && loss) e = hipMemcpy(loss, h->d_loss, sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_grad, 0, MLP_PARAMS * sizeof(float), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dfree(h, dD);
    dfree(h, dr);
    if (e != hipSuccess) return fail(h, CRMC_E_DEVICE, hipGetErrorString(e));
    return CRMC_OK;
}

int crmc_sweep(crmc_t h, double pH, double pKa, double mu_ion, int64_t n_sweeps)
{
    if (!h) return CRMC_E_ARG;
    std::vector<crmc_cond> c(h->reps.size());
    for (auto& x : c) {
        x.pH = pH; x.pKa = pKa; x.pKb = h->p.pKb; x.pIX_pos = mu_ion; x.pIX_neg = mu_ion; x.kappa = h->p.kappa;
    }
    return crmc_sweep_ex(h, c.data(), n_sweeps);
}

int crmc_observe(crmc_t h, int32_t replica, crmc_obs* out)
{
    if (!h || !out || replica < 0 || replica >= (int32_t)h->reps.size()) return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof *out);
    int64_t tot[4];
    uint64_t mv[14];
    std::vector<double> e(r.ncells);
    uint32_t err = 0;
    HIP_TRY(h, hipMemcpy(tot, r.d.totals, sizeof tot, hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(mv, r.d.moves, sizeof mv, hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(e.data(), r.d.e_acc, r.ncells * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(&err, h->d_err, sizeof err, hipMemcpyDeviceToHost));
    uint32_t hiw = 0;
    HIP_TRY(h, hipMemcpy(&hiw, r.d.hiwater, sizeof hiw, hipMemcpyDeviceToHost));
    double E = r.E0;
    for (double v : e) E += v;
    out->sweeps = h->sweeps;
    out->n_acid = r.nA;
    out->n_acid_charged = tot[0];
    out->n_base = r.nB;
    out->n_base_charged = tot[1];
    out->n_xpos = tot[2];
    out->n_xneg = tot[3];
    out->energy = E;
    for (int i = 0; i < 6; ++i) {
        out->attempts[i] = (int64_t)mv[i];
        out->accepts[i] = (int64_t)mv[6 + i];
    }
    out->relocation_attempts = (int64_t)mv[12];
    out->relocation_accepts = (int64_t)mv[13];
    out->error_flags = err;
    out->n_cells = (int32_t)r.n;
    out->cell_capacity = (int32_t)r.cap;
    out->max_cell_count = (int32_t)hiw;
    if (err & (ERR_BIN_CAPACITY | ERR_INSERT_CAPACITY))
        return fail(h, CRMC_E_CAPACITY, "a cell exceeded its record capacity; rebuild with a larger cell_capacity");
    return CRMC_OK;
}

int crmc_get_series(crmc_t h, int32_t replica, int64_t first, int64_t count, int32_t* out)
{
    if (!h || replica < 0 || replica >= (int32_t)h->reps.size() || count < 0 || (count && !out))
        return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    const int64_t capn = r.d.series_cap;
    if (first < 0 || first + count > h->sweeps || first < h->sweeps - capn)
        return fail(h, CRMC_E_ARG, "requested sweeps outside the retained window");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::vector<int32_t> all((size_t)capn * 4);
    HIP_TRY(h, hipMemcpy(all.data(), r.d.series, all.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) {
        const int64_t row = (first + i) % capn;
        std::memcpy(out + 4 * i, &all[(size_t)row * 4], 4 * sizeof(int32_t));
    }
    return CRMC_OK;
}

int crmc_get_particles(crmc_t h, int32_t replica, int32_t cap, uint32_t* xyz, int32_t* kind, int32_t* charged,
                       int32_t* site_id, int32_t* n_out)
{
    if (!h || replica < 0 || replica >= (int32_t)h->reps.size() || cap < 0 || !n_out)
        return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int buf = (int)(h->sweeps & 1);
    std::vector<uint32_t> cnt(r.ncells);
    std::vector<uint4> rec((size_t)r.ncells * r.cap);
    HIP_TRY(h, hipMemcpy(cnt.data(), r.d.cnt[buf], r.ncells * sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(rec.data(), r.d.rec[buf], rec.size() * sizeof(uint4), hipMemcpyDeviceToHost));
    int32_t k = 0;
    for (uint32_t c = 0; c < r.ncells; ++c)
        for (uint32_t j = 0; j < cnt[c]; ++j, ++k) {
            if (k >= cap) continue;
            const uint4 v = rec[(size_t)c * r.cap + j];
            if (xyz) { xyz[3 * k] = v.x; xyz[3 * k + 1] = v.y; xyz[3 * k + 2] = v.z; }
            const uint32_t sid = v.w >> 8;
            if (kind) kind[k] = (int32_t)(v.w & 7u);
            if (charged) charged[k] = (int32_t)((v.w >> 3) & 1u);
            if (site_id) site_id[k] = sid == NO_SITE ? -1 : (int32_t)sid;
        }
    *n_out = k;
    return check_device_errors(h);
}

int crmc_export_state(crmc_t h, void* buf, int64_t* bytes)
{
    if (!h || !bytes || (buf && *bytes < 0)) return fail(h, CRMC_E_ARG, "bad arguments");
    for (const HostReplica& r : h->reps)
        if (!r.built) return fail(h, CRMC_E_STATE, "every replica must be built before exporting the state");
    READY(h);
    Blob b;
    int rc = serialize_state(h, b);
    if (rc) return rc;
    const int64_t need = (int64_t)b.b.size();
    if (!buf) {
        *bytes = need;
        return CRMC_OK;
    }
    if (*bytes < need) {
        *bytes = need;
        return fail(h, CRMC_E_ARG, "state buffer too small (" + std::to_string(need) + " bytes needed)");
    }
    std::memcpy(buf, b.b.data(), (size_t)need);
    *bytes = need;
    return CRMC_OK;
}

int crmc_import_state(crmc_t h, const void* buf, int64_t bytes)
{
    if (!h || !buf || bytes <= 0) return fail(h, CRMC_E_ARG, "bad arguments");
    for (const HostReplica& r : h->reps)
        if (!r.built) return fail(h, CRMC_E_STATE, "build every replica from the same inputs before importing");
    READY(h);
    Cursor in{(const uint8_t*)buf, (size_t)bytes};
    const auto bad = [&](const char* what) { return fail(h, CRMC_E_ARG, std::string("state does not fit: ") + what); };
    char magic[8];
    uint32_t version = 0, nrep = 0, pad = 0;
    int32_t precision = 0;
    uint64_t seed = 0;
    int64_t sweeps = 0;
    if (!in.get_n(magic, 8) || std::memcmp(magic, STATE_MAGIC, 8) != 0) return bad("not a state");
    if (!in.get(version) || version != STATE_VERSION) return bad("unknown version");
    if (!in.get(nrep) || nrep != h->reps.size()) return bad("replica count");
    if (!in.get(precision) || precision != h->p.precision) return bad("precision");
    if (!in.get(pad) || !in.get(seed) || seed != h->p.seed) return bad("seed");
    if (!in.get(sweeps) || sweeps < 0 || (uint64_t)sweeps >= (1ull << 32)) return bad("sweep counter");
    uint64_t md_steps = 0;
    if (!in.get(md_steps)) return bad("truncated");

    // parse everything on the host first; the handle changes only if all of it fits
    struct RepState {
        double E0, e0_kappa;
        uint32_t hiw;
        std::vector<uint32_t> cnt;
        std::vector<uint4> rec;
        std::vector<double> e;
        std::vector<uint64_t> occ;
        std::vector<int32_t> gc, series;
        std::vector<int64_t> gh;
        int64_t tot[4];
        uint64_t mv[14];
        double lp_off[2];
    };
    std::vector<RepState> st(nrep);
    for (uint32_t i = 0; i < nrep; ++i) {
        const HostReplica& r = h->reps[i];
        RepState& q = st[i];
        RepShape sh{};
        uint32_t pad2 = 0;
        if (!in.get(sh) || !same_shape(sh, shape_of(r))) return bad("replica geometry");
        if (!in.get(q.E0) || !in.get(q.e0_kappa) || !in.get(q.hiw) || !in.get(pad2)) return bad("truncated");
        q.cnt.resize(r.ncells);
        if (!in.get_n(q.cnt.data(), q.cnt.size())) return bad("truncated");
        q.rec.assign((size_t)r.ncells * r.cap, make_uint4(0, 0, 0, 0));
        for (uint32_t c = 0; c < r.ncells; ++c) {
            if (q.cnt[c] > r.cap) return bad("cell count above capacity");
            if (!in.get_n(&q.rec[(size_t)c * r.cap], q.cnt[c])) return bad("truncated");
        }
        q.e.resize(r.ncells);
        q.occ.resize(r.nsites);
        q.gc.resize(2 * std::max<uint32_t>(r.ngroups, 1));
        q.gh.resize((size_t)r.hist_off[r.ngroups]);
        if (!in.get_n(q.e.data(), q.e.size()) || !in.get_n(q.occ.data(), q.occ.size()) ||
            !in.get_n(q.gc.data(), q.gc.size()) || !in.get_n(q.gh.data(), q.gh.size()) || !in.get_n(q.tot, 4) ||
            !in.get_n(q.mv, 14))
            return bad("truncated");
        int64_t capn = 0;
        if (!in.get(capn) || capn != r.d.series_cap) return bad("series window");
        const int64_t rows = std::min<int64_t>(sweeps, capn);
        q.series.resize((size_t)rows * 4);
        if (!in.get_n(q.series.data(), q.series.size()) || !in.get_n(q.lp_off, 2)) return bad("truncated");
    }
    uint32_t learned = 0, has_par = 0;
    double eps = 0.0;
    std::vector<float> w, m, v;
    int64_t adam_t = 0;
    if (!in.get(learned) || !in.get(eps) || !in.get(has_par) || learned > 1 || has_par > 1) return bad("proposal");
    if (learned && (!(eps > 0.0) || eps > 1.0)) return bad("proposal eps");
    if (has_par) {
        w.resize(MLP_PARAMS);
        m.resize(MLP_PARAMS);
        v.resize(MLP_PARAMS);
        if (!in.get_n(w.data(), w.size()) || !in.get_n(m.data(), m.size()) || !in.get_n(v.data(), v.size()) ||
            !in.get(adam_t))
            return bad("truncated network");
    }
    if (in.at != in.n) return bad("trailing bytes");

    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int buf_now = (int)(sweeps & 1);
    for (uint32_t i = 0; i < nrep; ++i) {
        HostReplica& r = h->reps[i];
        const RepState& q = st[i];
        Replica& d = r.d;
        HIP_TRY(h, hipMemcpy(d.rec[buf_now], q.rec.data(), q.rec.size() * sizeof(uint4), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.cnt[buf_now], q.cnt.data(), q.cnt.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemset(d.cnt[buf_now ^ 1], 0, r.ncells * sizeof(uint32_t)));
        HIP_TRY(h, hipMemcpy(d.e_acc, q.e.data(), q.e.size() * sizeof(double), hipMemcpyHostToDevice));
        if (r.nsites)
            HIP_TRY(h, hipMemcpy(d.occupancy, q.occ.data(), q.occ.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.group_count, q.gc.data(), q.gc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        if (!q.gh.empty())
            HIP_TRY(h, hipMemcpy(d.group_hist, q.gh.data(), q.gh.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.totals, q.tot, sizeof q.tot, hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.moves, q.mv, sizeof q.mv, hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.hiwater, &q.hiw, sizeof q.hiw, hipMemcpyHostToDevice));
        std::vector<int32_t> all((size_t)d.series_cap * 4, 0);
        const int64_t first = std::max<int64_t>(0, sweeps - d.series_cap);
        for (int64_t s = first; s < sweeps; ++s)
            std::memcpy(&all[(size_t)(s % d.series_cap) * 4], &q.series[(size_t)(s - first) * 4], 4 * sizeof(int32_t));
        HIP_TRY(h, hipMemcpy(d.series, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        // the cached grid shifts are recomputed from the sweep counter
        HIP_TRY(h, hipMemset(d.tab, 0, sizeof(SweepTab)));
        d.lp_off[0] = q.lp_off[0];
        d.lp_off[1] = q.lp_off[1];
        r.E0 = q.E0;
        r.e0_kappa = q.e0_kappa;
    }
    const uint64_t s64 = (uint64_t)sweeps;
    HIP_TRY(h, hipMemcpy(h->d_sweep, &s64, sizeof s64, hipMemcpyHostToDevice));
    h->sweeps = sweeps;
    h->md_steps = md_steps;
    h->learned = learned != 0;
    h->learn_eps = eps;
    if (has_par) {
        int rc = ensure_params(h);
        if (rc) return rc;
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        HIP_TRY(h, hipMemcpy(h->d_p32, w.data(), MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_adam_m, m.data(), MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_adam_v, v.data(), MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
        h->adam_t = adam_t;
        LearnArgs g = learn_args(h);
        HIP_TRY(h, launch_params_convert(g, h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return CRMC_OK;
}

int crmc_energy(crmc_t h, int32_t replica, double* out)
{
    if (!h || !out || replica < 0 || replica >= (int32_t)h->reps.size()) return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    return state_energy(h, r, out);
}

int crmc_energy_noalloc(crmc_t h, int32_t replica, double* out)
{
    if (!h || !out || replica < 0 || replica >= (int32_t)h->reps.size()) return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    if (!r.on_device)
        return fail(h, CRMC_E_STATE, "the replica's device state does not exist yet (it would have to be allocated)");
    if ((size_t)r.ncells > NOALLOC_CELLS)
        return fail(h, CRMC_E_ARG, "more cells than the fixed scratch holds (" + std::to_string(NOALLOC_CELLS) + ")");
    void* base = nullptr;
    HIP_TRY(h, noalloc_scratch(&base));
    Replica* d_rep = (Replica*)base;
    double* d_e = (double*)((char*)base + NOALLOC_DESC_BYTES);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpyAsync(d_rep, &r.d, sizeof(Replica), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_energy(d_rep, r.d, h->p.lB, h->p.eps_wca, h->p.ion_coupling, (int)(h->sweeps & 1), d_e,
                             h->stream));
    // the per-cell sums, added on the host in cell order (as crmc_energy does)
    double chunk[2048];
    double E = 0.0;
    for (size_t c0 = 0; c0 < r.ncells; c0 += 2048) {
        const size_t m = std::min<size_t>(2048, r.ncells - c0);
        HIP_TRY(h, hipMemcpyAsync(chunk, d_e + c0, m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (size_t i = 0; i < m; ++i) E += chunk[i];
    }
    *out = E;
    return CRMC_OK;
}

int crmc_ungroup(crmc_t h, int32_t replica, const double frac[4], uint64_t draw, int64_t counts[6],
                 int8_t* labels, int64_t cap, int64_t* n_out)
{
    if (!h || !frac || !counts || replica < 0 || replica >= (int32_t)h->reps.size() || cap < 0 || (cap && !labels))
        return fail(h, CRMC_E_ARG, "bad arguments");
    for (int i = 0; i < 4; ++i)
        if (!(frac[i] >= 0.0) || frac[i] > 1.0) return fail(h, CRMC_E_ARG, "fractions must lie in [0, 1]");
    if (frac[0] + frac[1] > 1.0 + 1e-12 || frac[2] + frac[3] > 1.0 + 1e-12)
        return fail(h, CRMC_E_ARG, "the subspecies fractions of one sign sum to more than 1");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int buf = (int)(h->sweeps & 1);
    std::vector<uint32_t> cnt(r.ncells), pre(r.ncells);
    HIP_TRY(h, hipMemcpy(cnt.data(), r.d.cnt[buf], r.ncells * sizeof(uint32_t), hipMemcpyDeviceToHost));
    uint32_t np = 0;
    for (uint32_t c = 0; c < r.ncells; ++c) { pre[c] = np; np += cnt[c]; }
    if (n_out) *n_out = np;
    Replica* d_rep = nullptr;
    uint32_t* d_pre = nullptr;
    int8_t* d_lab = nullptr;
    unsigned long long* d_cnt = nullptr;
    hipError_t e = dalloc(h, &d_rep, 1);
    if (e == hipSuccess) e = dalloc(h, &d_pre, r.ncells);
    if (e == hipSuccess && cap) e = dalloc(h, &d_lab, (size_t)std::max<uint32_t>(np, 1));
    if (e == hipSuccess) e = dalloc(h, &d_cnt, 6);
    if (e == hipSuccess) e = hipMemcpy(d_rep, &r.d, sizeof(Replica), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_pre, pre.data(), r.ncells * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_cnt, 0, 6 * sizeof(unsigned long long));
    if (e == hipSuccess) e = launch_ungroup(d_rep, r.d, buf, d_pre, frac, draw, d_lab, d_cnt, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    unsigned long long cc[6] = {0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(cc, d_cnt, sizeof cc, hipMemcpyDeviceToHost);
    if (e == hipSuccess && cap && np)
        e = hipMemcpy(labels, d_lab, std::min<size_t>((size_t)cap, np) * sizeof(int8_t), hipMemcpyDeviceToHost);
    dfree(h, d_rep);
    dfree(h, d_pre);
    dfree(h, d_lab);
    dfree(h, d_cnt);
    if (e != hipSuccess)
        return fail(h, e == hipErrorOutOfMemory ? CRMC_E_NOMEM : CRMC_E_DEVICE, std::string("ungrouping: ") + hipGetErrorString(e));
    for (int i = 0; i < 6; ++i) counts[i] = (int64_t)cc[i];
    return CRMC_OK;
}

int crmc_get_occupancy(crmc_t h, int32_t replica, int64_t cap, uint64_t* out, int64_t* n_out)
{
    if (!h || !n_out || replica < 0 || replica >= (int32_t)h->reps.size() || cap < 0)
        return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    *n_out = r.nsites;
    const int64_t m = std::min<int64_t>(cap, r.nsites);
    if (m > 0) HIP_TRY(h, hipMemcpy(out, r.d.occupancy, (size_t)m * sizeof(uint64_t), hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_get_group_hist(crmc_t h, int32_t replica, int64_t cap, int64_t* out, int32_t off_cap, int32_t* off,
                        int32_t* n_groups)
{
    if (!h || !n_groups || replica < 0 || replica >= (int32_t)h->reps.size() || cap < 0 || off_cap < 0)
        return fail(h, CRMC_E_ARG, "bad arguments");
    HostReplica& r = h->reps[(size_t)replica];
    if (!r.built) return fail(h, CRMC_E_STATE, "replica not built");
    READY(h);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    *n_groups = (int32_t)r.ngroups;
    for (int32_t i = 0; i < std::min<int32_t>(off_cap, (int32_t)r.ngroups + 1); ++i) off[i] = r.hist_off[(size_t)i];
    const int64_t m = std::min<int64_t>(cap, r.hist_off[r.ngroups]);
    if (m > 0) HIP_TRY(h, hipMemcpy(out, r.d.group_hist, (size_t)m * sizeof(int64_t), hipMemcpyDeviceToHost));
    return CRMC_OK;
}

int crmc_enable_log(crmc_t h, int64_t capacity)
{
    if (!h || capacity < 0) return fail(h, CRMC_E_ARG, "bad arguments");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    dfree(h, h->d_log);
    h->d_log = nullptr;
    if (!h->d_log_n) HIP_TRY(h, dalloc(h, &h->d_log_n, 1));
    HIP_TRY(h, hipMemset(h->d_log_n, 0, sizeof(unsigned long long)));
    h->log_cap = capacity;
    if (capacity > 0) HIP_TRY(h, dalloc(h, &h->d_log, (size_t)capacity));
    return CRMC_OK;
}

int crmc_read_log(crmc_t h, int64_t cap, crmc_trial_rec* out, int64_t* n_out)
{
    static_assert(sizeof(crmc_trial_rec) == sizeof(TrialRec), "trial record layout");
    if (!h || !n_out || cap < 0) return fail(h, CRMC_E_ARG, "bad arguments");
    *n_out = 0;
    if (!h->d_log) return CRMC_OK;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    unsigned long long n = 0;
    HIP_TRY(h, hipMemcpy(&n, h->d_log_n, sizeof n, hipMemcpyDeviceToHost));
    const int64_t m = std::min<int64_t>({(int64_t)n, h->log_cap, cap});
    if (m > 0) HIP_TRY(h, hipMemcpy(out, h->d_log, (size_t)m * sizeof(TrialRec), hipMemcpyDeviceToHost));
    *n_out = (int64_t)n;
    return CRMC_OK;
}

int crmc_enable_trace(crmc_t h, int64_t capacity)
{
    static_assert(sizeof(crmc_phase_trace) == sizeof(PhaseTrace), "trace record layout");
    if (!h || capacity < 0) return fail(h, CRMC_E_ARG, "bad arguments");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    dfree(h, h->d_trace);
    h->d_trace = nullptr;
    if (!h->d_trace_n) HIP_TRY(h, dalloc(h, &h->d_trace_n, 1));
    HIP_TRY(h, hipMemset(h->d_trace_n, 0, sizeof(unsigned long long)));
    h->trace_cap = capacity;
    if (capacity > 0) HIP_TRY(h, dalloc(h, &h->d_trace, (size_t)capacity));
    return CRMC_OK;
}

int crmc_read_trace(crmc_t h, int64_t cap, crmc_phase_trace* out, int64_t* n_out)
{
    if (!h || !n_out || cap < 0) return fail(h, CRMC_E_ARG, "bad arguments");
    *n_out = 0;
    if (!h->d_trace) return CRMC_OK;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    unsigned long long n = 0;
    HIP_TRY(h, hipMemcpy(&n, h->d_trace_n, sizeof n, hipMemcpyDeviceToHost));
    const int64_t m = std::min<int64_t>({(int64_t)n, h->trace_cap, cap});
    if (m > 0) HIP_TRY(h, hipMemcpy(out, h->d_trace, (size_t)m * sizeof(PhaseTrace), hipMemcpyDeviceToHost));
    *n_out = (int64_t)n;
    return CRMC_OK;
}

int crmc_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out)
{
    if (n < 0 || (n > 0 && (!ctr || !out))) return CRMC_E_ARG;
    if (n == 0) return CRMC_OK;
    uint32_t *dc = nullptr, *dout = nullptr;
    if (hipMalloc((void**)&dc, (size_t)n * 16) != hipSuccess) return CRMC_E_NOMEM;
    if (hipMalloc((void**)&dout, (size_t)n * 16) != hipSuccess) { (void)hipFree(dc); return CRMC_E_NOMEM; }
    int rc = CRMC_OK;
    if (hipMemcpy(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice) != hipSuccess ||
        launch_philox(n, dc, k0, k1, dout, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost) != hipSuccess)
        rc = CRMC_E_DEVICE;
    (void)hipFree(dc);
    (void)hipFree(dout);
    return rc;
}

int crmc_set_timing(crmc_t h, int32_t on)
{
    if (!h) return CRMC_E_ARG;
    int rc = drain_timing(h, 0);
    if (rc) return rc;
    h->timing = on != 0;
    for (int i = 0; i < 3; ++i) { h->t_ms[i] = 0.0; h->t_n[i] = 0; }
    return CRMC_OK;
}

int crmc_get_timing(crmc_t h, double ms[3], int64_t launches[3])
{
    if (!h || !ms || !launches) return fail(h, CRMC_E_ARG, "bad arguments");
    int rc = drain_timing(h, 0);
    if (rc) return rc;
    for (int i = 0; i < 3; ++i) { ms[i] = h->t_ms[i]; launches[i] = h->t_n[i]; }
    return CRMC_OK;
}

void crmc_destroy(crmc_t h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (auto& p : h->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : h->free_events) (void)hipEventDestroy(e);
    if (h->gstream) (void)hipStreamSynchronize(h->gstream);
    drop_graphs(h);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    for (auto& r : h->reps)
        if (r.built) free_replica(h, r);
    dfree(h, h->d_reps);
    dfree(h, h->d_sweep);
    dfree(h, h->d_err);
    dfree(h, h->d_log);
    dfree(h, h->d_log_n);
    dfree(h, h->d_trace);
    dfree(h, h->d_trace_n);
    dfree(h, h->d_cell2rep);
    dfree(h, h->d_dom2rep);
    dfree(h, h->d_lntab);
    dfree(h, h->d_plan_n);
    dfree(h, h->d_plan_heavy);
    dfree(h, h->d_plan_light);
    dfree(h, h->d_plan_geo_heavy);
    dfree(h, h->d_plan_geo_light);
    void* lp[] = {h->d_R2sh, h->d_p32, h->d_p64, h->d_w1b, h->d_w2b, h->d_adam_m, h->d_adam_v,
                  h->d_grad, h->d_loss, h->d_data, h->d_data_n, h->d_lwork, h->d_md_vel, h->d_md_force};
    for (void* q : lp) dfree(h, q);
    delete h;
}

} // extern "C"
