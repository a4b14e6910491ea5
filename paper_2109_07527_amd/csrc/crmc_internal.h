// Internal definitions shared by the host library and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crmc {

constexpr uint32_t KIND_ACID = 1, KIND_BASE = 2, KIND_XPOS = 3, KIND_XNEG = 4, KIND_NEUTRAL = 5;
constexpr uint32_t TAG_TRIAL = 1, TAG_SHIFT = 2, TAG_PAIR = 4, TAG_UNGROUP = 5;
constexpr uint32_t NO_SITE = 0xFFFFFFu;

constexpr uint32_t ERR_BIN_CAPACITY = 1u;
constexpr uint32_t ERR_INSERT_CAPACITY = 2u;
constexpr uint32_t INFO_UNSTAGED = 4u;   // some neighbours were read from memory during trials
constexpr uint32_t ERR_POOL = 8u;        // a domain did not fit its LDS pool (not processed)

// A phase's thousands of domains add their counts to 256 copies of a
// replica's counters (one per 128-byte line) rather than to one line; a
// sweep's counts fit in 32 bits
constexpr int CTR_STRIPES = 256, CTR_STRIDE = 32;

constexpr int BIN_THREADS = 256;    // four wavefronts
// new cells per wavefront of the re-binning: BIN_CPW once a launch has
// enough cells to fill the chip that way, else one
constexpr uint32_t BIN_CPW = 8, BIN_BATCH_MIN_CELLS = 65536;
constexpr int PHASE_THREADS = 256;  // one heavy domain, or four light domains (one per wavefront)
constexpr int DEFAULT_LIGHT_NB = 768;

// sweep plan counters (cleared by the re-binning kernel), one 128-byte line
// per colour: heavy domains, light domains, work items of the feature kernel
constexpr int PLAN_STRIDE = 32, PLAN_HEAVY = 0, PLAN_LIGHT = 1, PLAN_LWORK = 2;
constexpr int PLAN_N = 8 * PLAN_STRIDE;
__host__ __device__ constexpr int plan_idx(int colour, int k) { return colour * PLAN_STRIDE + k; }

// learned proposal network: W1[128][32], b1[128], W2[128][128], b2[128], w3[128], b3
constexpr int MLP_IN = 32, MLP_H = 128;
constexpr int MLP_B1 = MLP_H * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_H;
constexpr int MLP_PARAMS = MLP_B3 + 1;

// Record: three fixed-point coordinates and a meta word
//   bits 0-2 kind, bit 3 charged flag, bits 8-31 site id (NO_SITE for ions)
__host__ __device__ inline uint32_t make_meta(uint32_t kind, uint32_t charged, uint32_t sid)
{
    return kind | (charged << 3) | (sid << 8);
}

// per replica, rewritten by the re-binning kernel every sweep
struct SweepTab {
    uint32_t o[4];     // grid shift of the current sweep
    uint32_t pairc[8]; // reflection centre of the active-cell pairing, per colour
    // written at the end of a sweep for the next one: its shift and the one
    // it follows, valid for sweep number valid - 1 (0: none)
    uint32_t next[4], prev[4];
    uint64_t valid;
};

// One replica as the kernels see it.
struct Replica {
    uint4* rec[2];           // ping-pong record buffers, ncells*cap records each
    uint32_t* cnt[2];        // records per cell
    uint32_t* cnt0;          // records per cell as binned at the start of the sweep
    double* e_acc;           // per cell: accumulated energy change of accepted trials
    uint64_t* occupancy;     // per site: sweeps at whose start it was charged
    int32_t* site_group;     // per site: group index
    int32_t* group_count;    // 2 x ngroups: ionized sites per group at sweep start (by parity)
    int64_t* group_hist;     // per group histogram of ionized-site counts
    int32_t* group_hist_off; // ngroups+1 offsets into group_hist
    uint4* core_x;           // core centres (x, y, z, unused)
    double* core_delta;      // Delta = R - 1/2
    int64_t* totals;         // nA-, nB+, nX+, nX-
    uint64_t* moves;         // attempts[6], accepts[6], relocation attempts and accepts
    uint32_t* ctr;           // CTR_STRIPES stripes of CTR_STRIDE: one sweep's adds of the domains
                             // to moves (0-13) and totals (14-17, two's complement), folded into
                             // them and cleared at the end of every sweep
    int32_t* series;         // series_cap rows of 4
    uint32_t* bnd;           // n+1 cell boundaries b_k = ceil(k 2^32 / n), b_n stored as 0
    double* lnW;             // n: ln of the cell widths in lattice units
    uint32_t* hiwater;       // largest cell count seen by the re-binning
    SweepTab* tab;
    int64_t series_cap;
    uint32_t n, h, ncells, cap;
    uint32_t ncores, nsites, ngroups;
    uint32_t key0, key1;
    uint32_t cell_begin;     // prefix of cells over replicas (binning grid)
    uint32_t dom_begin;      // prefix of domains per phase over replicas
    uint32_t* nsc;           // per cell: acid and base sites as binned at the start of the sweep
    uint32_t bin_sparse;     // 1: re-binned one lane per cell (far fewer particles than cells)
    double* phat;            // per site: network output of the current phase (learned proposal)
    float* feat;             // per site: its 32 features as last evaluated (only while recording; else null)
    double lp_off[2];        // logit offsets of acid and base sites (learned proposal)
    double L, scale, lnZ0;   // scale = L / 2^32; lnZ0 = ln(rho0 NA) + 3 ln(scale)
    uint64_t R2;             // Coulomb cutoff on the integer squared distance
    double lnKA, lnKB, lnKion, kappa;
};

struct TrialRec {
    int64_t sweep, cell;
    int32_t trial, replica;
    int32_t move, status;
    double dU, lnp, u;
};

// optional per-workgroup trace of the phase kernel (profiling)
struct PhaseTrace {
    uint64_t t0, t1;        // wall clock at start and end of the workgroup
    uint32_t sweep, domain; // sweep, global domain index
    int32_t colour, ntr;    // colour, trials run
    int32_t nb, own;        // neighbour records, records in the domain's cells
    int32_t staged, hw;     // neighbours staged on chip; hardware id of the wave
};

struct SweepArgs {
    Replica* reps;
    const uint32_t* cell2rep; // global cell index -> replica
    const uint32_t* dom2rep;  // global domain index (of one phase) -> replica
    const double* lntab;      // ln k for k < lntab_n (k = 0 unused)
    int32_t lntab_n;
    uint32_t nrep;
    uint32_t ncell_total;
    uint32_t ndom_total;
    int32_t colour;
    uint64_t* sweep;   // device sweep counter (all replicas advance together)
    uint32_t* err;     // device error flags
    TrialRec* log;
    unsigned long long* log_n;
    uint64_t log_cap;
    double lB, eps, ln2;
    int32_t ion_coupling, trials, pairing, fixed_grid, site_trials;
    int32_t ion_trials; // ion relocation trials per cell of a domain, after the reaction trials
    int32_t bin_sparse_any; // some replica is re-binned one lane per cell
    int32_t bin_dense_any;  // some replica is re-binned by wavefronts (k_bin)
    int32_t bin_cpw;        // new cells per wavefront of k_bin
    int32_t pool;      // LDS pool of a phase workgroup, in records (a light domain gets a quarter)
    int32_t precision; // 32 or 64
    int32_t light_nb;  // neighbour records up to which a domain may run on one wavefront
    uint32_t* plan_n;      // plan_idx(c, PLAN_HEAVY / PLAN_LIGHT / PLAN_LWORK): heavy and light
                           // domains of colour c, work items of the learned proposal's feature kernel
    uint32_t* plan_heavy;  // per colour: ndom_total slots of domain indices
    uint32_t* plan_light;
    uint4* plan_geo_heavy; // beside each slot: replica, first and second cell, and
    uint4* plan_geo_light; // the two cells' binned counts (16 bits each)
    struct LearnItem* lwork; // per colour: lwork_cap work items of the feature kernel, or null
                             // when no learned-proposal kernel runs
    uint32_t lwork_cap;
    int32_t learned;   // site picks by the learned proposal
    double learn_eps;  // weight of the uniform pick in it
    PhaseTrace* trace;
    unsigned long long* trace_n;
    uint64_t trace_cap;
};

// A work item of the feature kernel: sites 64 part .. 64 part + 63 of one
// cell, with what the kernel needs of the replica resolved for the sweep
struct LearnItem {
    const uint4* rec;      // the sweep's record buffer of the replica
    const uint32_t* cnt;   // its cell counts
    double* phat;          // per site network outputs
    float* feat;           // per site features (recording only; else null)
    double off[2];         // logit offsets of acid and base sites
    uint32_t cell, part, r, n, cap, pad;
};

// arguments of the learned-proposal kernels
struct LearnArgs {
    uint32_t grid;            // workgroups of the feature kernel (they stride over the work items)
    const uint64_t* R2sh;     // per replica: 17 shell thresholds on the squared lattice distance
    float* p32;               // FP32 master parameters
    double* p64;              // FP64 copy (FP64 inference)
    short* w1b;               // BF16 W1 [128][32]
    short* w2b;               // BF16 W2 [128][128]
    float* data;              // training rows: 32 features + label
    unsigned long long* data_n;
    uint64_t data_cap;
    int32_t infer;            // compute site probabilities (else features / rows only)
};

// arguments of the molecular-dynamics kernels (hybrid MD / CR-MC)
struct MdArgs {
    Replica* reps;            // device replica descriptors
    const uint32_t* cell2rep; // global cell index -> replica
    uint32_t ncell_total;
    double* const* vel;       // per replica and record buffer (2 r + buf): 3 doubles per record slot
    double* const* force;     // per replica: 3 doubles per record slot of the current buffer
    uint32_t* err;            // device error flags
    double lB, eps, dt, gamma, noise; // noise = sqrt(2 gamma kT / (m dt)), kT = m = 1
    int32_t ion_coupling;
    int32_t precision;        // 32: pair forces in FP32 (summed in FP64), 64: all FP64
};

// launchers (device translation units)
hipError_t launch_bin(const SweepArgs& a, hipStream_t s);
hipError_t launch_plan(const SweepArgs& a, hipStream_t s);
hipError_t launch_phase(const SweepArgs& a, size_t lds_bytes, hipStream_t s);
hipError_t launch_sweep_end(const SweepArgs& a, hipStream_t s);
// fixed scratch of crmc_energy_noalloc (see noalloc_scratch)
constexpr size_t NOALLOC_DESC_BYTES = 1024;
constexpr size_t NOALLOC_CELLS = (size_t)1 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(void** out);
hipError_t launch_ungroup(const Replica* rep_dev, const Replica& rep_host, int buf, const uint32_t* prefix,
                          const double frac[4], uint64_t draw, int8_t* labels, unsigned long long* counts,
                          hipStream_t s);
hipError_t launch_energy(const Replica* rep_dev, const Replica& rep_host, double lB, double eps,
                         int ion_coupling, int buf, double* out_per_cell, hipStream_t s);
hipError_t launch_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                         hipStream_t s);
hipError_t set_phase_lds_limit(size_t bytes);
hipError_t launch_learn(const SweepArgs& a, const LearnArgs& g, hipStream_t s);
hipError_t launch_mlp_fwd(const LearnArgs& g, const float* X, int nrows, float* out, hipStream_t s);
hipError_t launch_mlp_grad(const LearnArgs& g, const float* data, const int* rows, int nrows, float inv_batch,
                           float* grad, double* loss, hipStream_t s);
hipError_t launch_adam(const LearnArgs& g, float* grad, float* m, float* v, float lr, float c1, float c2,
                       hipStream_t s);
hipError_t launch_params_convert(const LearnArgs& g, hipStream_t s);
hipError_t set_learn_lds_limit();
hipError_t launch_md_block(const MdArgs& m, int buf0, uint64_t step0, int64_t nsteps, uint32_t maxcap, hipStream_t s,
                           int* buf_out);

} // namespace crmc
