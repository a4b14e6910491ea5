/*
 * crmc.h - C ABI of the MI355X charge-regulation Monte Carlo (CR-MC) library.
 *
 * The method is the one of Curk, Yuan and Luijten, "Accelerated simulation
 * method for charge regulation effects": acid and base groups ionize by the
 * grouped reactions A <-> A- + X+, B <-> B+ + X-, and salt pairs enter and
 * leave by 0 <-> X+ + X- (Sec. II B).  Each trial is one of the six moves
 * (forward/reverse of each reaction, equal probability), picks its
 * participants uniformly, computes the energy change from the changed
 * particles only and accepts with the Metropolis probabilities of Sec. II C,
 * written with pH, pOH = pKw - pH, pK and the combined-ion chemical potentials
 * pI_X+ / pI_X- in log10 units (eq. pIXgen gives pI_X from a salt pI_S).
 *
 * Parallel schedule.  Each sweep draws a random shift of a cubic cell grid
 * (cell width >= cutoff, an even number >= 4 of cells per edge) and re-bins all
 * particles into the shifted cells.  The cells are split into 8 parity classes
 * (colours); cells of one colour never interact, so all of them are updated at
 * once.  In the phase of a colour the active cells are paired by a random
 * reflection of their index; a trial acts on such a pair ("domain"): it picks
 * participants among the domain's particles and inserts ions uniformly in one
 * of its two cells, with the paper's acceptance probability in which the volume
 * is the insertion volume of the domain and every count is the domain's count.
 * With pairing off a domain is a single cell.
 *
 * Energy model (units: length sigma, energy kT):
 *   screened Coulomb lB q_i q_j exp(-kappa r)/r for r < rc (truncated),
 *   excluded volume 4 eps (r^-12 - r^-6) + eps for r < 2^(1/6) between a free
 *   ion and any other particle (Table I, eq. LJ with C = 1/4),
 *   expanded excluded volume between a free ion and a nanoparticle core of
 *   radius R with Delta = R - 1/2 (Table II, eq. LJe).
 * A free ion closer than 1/2 to a particle (or than Delta + 1/2 to a core
 * centre) is an overlap and is never accepted.  Positions are 32-bit fixed
 * point per box edge; the Coulomb cutoff is decided exactly on the integer
 * squared distance.
 *
 * Conventions.
 *   - Every host array passed in is owned by the caller and copied before the
 *     call returns; the library never frees caller memory.
 *   - Device memory: every buffer of a handle's state comes either from the
 *     library (hipMalloc, freed by crmc_destroy) or, when the caller hands one
 *     over (crmc_params.workspace, or crmc_set_workspace right after the
 *     builds), from a caller-owned workspace such as a torch uint8 tensor;
 *     then the handle never allocates device memory of its own and
 *     crmc_destroy frees nothing of it.  crmc_build_cells keeps a replica's
 *     initial state on the host; the device state is created by the first
 *     call that needs it.
 *   - Calls that launch work are asynchronous and ordered on the stream given
 *     in crmc_params (NULL = the default stream).  crmc_observe,
 *     crmc_get_series, crmc_get_particles, crmc_energy, crmc_read_log,
 *     crmc_export_state, crmc_import_state and crmc_destroy synchronize.
 *   - Errors: a negative status; crmc_last_error() describes the last one.
 *     Device-side conditions (a cell running out of capacity) are reported as
 *     CRMC_E_CAPACITY by the next synchronizing call; the state is then not
 *     trustworthy.  No C++ exception crosses the ABI.  A handle is not
 *     thread-safe.
 */
#ifndef CRMC_H
#define CRMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CRMC_ABI_VERSION 3

typedef struct crmc_s* crmc_t;

enum crmc_status {
    CRMC_OK = 0,
    CRMC_E_ARG = -1,      /* invalid argument */
    CRMC_E_NOMEM = -2,    /* device or host allocation failed */
    CRMC_E_DEVICE = -3,   /* HIP runtime error */
    CRMC_E_CAPACITY = -4, /* a cell exceeded its record capacity */
    CRMC_E_STATE = -5     /* call out of order (e.g. sweep before build) */
};

/* particle kinds (sites keep their kind; their ionization is a separate flag) */
enum crmc_kind {
    CRMC_ACID = 1,    /* A (neutral) / A- (charged, q = -1) */
    CRMC_BASE = 2,    /* B (neutral) / B+ (charged, q = +1) */
    CRMC_XPOS = 3,    /* free monovalent cation X+ */
    CRMC_XNEG = 4,    /* free monovalent anion X- */
    CRMC_NEUTRAL = 5  /* non-ionizable bead (excluded volume for ions only) */
};

/* move ids used by statistics and trial logs */
enum crmc_move {
    CRMC_ACID_FWD = 0, CRMC_ACID_BACK = 1, CRMC_BASE_FWD = 2,
    CRMC_BASE_BACK = 3, CRMC_SALT_IN = 4, CRMC_SALT_OUT = 5,
    CRMC_ION_RELOCATE = 6 /* not one of the paper's moves: see crmc_params.ion_trials */
};

typedef struct {
    int32_t n_replicas;      /* independent systems advanced together (>= 1) */
    int32_t precision;       /* 32: pair terms in FP32 (FP64 sums); 64: all FP64 */
    int32_t trials_per_cell; /* trials per active cell per phase (>= 1) */
    int32_t pairing;         /* 1: domains are reflection-paired cells; 0: single cells */
    int32_t ion_coupling;    /* 1: ions interact; 0: ideal ions (test systems) */
    int32_t lds_records;     /* LDS pool of a phase workgroup in 16-byte records (0 = 4096); raised
                                to 3 * cell_capacity + 128 when smaller.  A heavy domain has the
                                whole pool, a light domain a quarter of it */
    int32_t fixed_grid;      /* 1: never shift the grid (only for tests: not ergodic) */
    int32_t site_trials;     /* extra trials per 16 ionizable sites of a domain (rounded up) */
    int32_t light_neighbours; /* a domain whose 26-cell neighbourhoods held at most this many
                                 records at the start of the sweep, and whose lists fit a quarter
                                 of the pool, runs on one wavefront; the others on a whole
                                 256-thread workgroup (0 = 768; 1..65536).  Results do not
                                 depend on it */
    int32_t use_graph;       /* 1: replay captured HIP graphs of whole sweeps; 0: launch each kernel */
    int32_t learned_proposal; /* 1: acid/base sites picked by the learned proposal (see
                                 crmc_set_proposal); 0: uniform picks */
    int32_t ion_trials;      /* ion relocation trials per cell of a domain per phase, after the
                                reaction trials (0 = none, the paper's six moves only; <= 4096).
                                A relocation (move id 6) removes a free ion of the domain picked
                                uniformly (cations first in the ordering) and re-inserts it at a
                                point drawn like an insertion of its sign, accepted with
                                min(1, (V_new / V_old) exp(-dU)), V the insertion volume of the
                                cell drawn.  It stands in for the ion motion the paper gets from
                                molecular dynamics: the six moves alone move an ion only by
                                deleting and re-inserting it with a reaction, which mixes ion
                                positions very slowly when salt is dilute */
    double lB;               /* Bjerrum length (sigma) */
    double rc;               /* Coulomb cutoff (sigma) */
    double eps_wca;          /* excluded-volume strength (kT); 0 disables it */
    double rho0NA;           /* reference density rho0 NA in sigma^-3 (rho0 = 1 M) */
    double pKw;              /* water: pOH = pKw - pH */
    double kappa;            /* default inverse screening length (sigma^-1) */
    double pKb;              /* default base pK used by crmc_sweep */
    double learned_eps;      /* weight of the uniform pick in the learned proposal, in (0, 1] */
    uint64_t seed;           /* Philox key: (seed low word, seed high word ^ replica) */
    void* stream;            /* hipStream_t on which every call is ordered */
    void* workspace;         /* caller-owned device memory for the handle's state, or NULL (the
                                library allocates); it must stay valid until crmc_destroy */
    int64_t workspace_bytes; /* its size (>= 256 when workspace is set); see crmc_workspace_size */
} crmc_params;

/* Per-replica reservoir conditions for crmc_sweep_ex. */
typedef struct {
    double pH, pKa, pKb;     /* pOH = pKw - pH */
    double pIX_pos, pIX_neg; /* combined-ion chemical potentials (log10 units) */
    double kappa;            /* inverse screening length of this replica */
} crmc_cond;

typedef struct {
    int64_t sweeps;           /* sweeps done since build */
    int64_t n_acid, n_acid_charged, n_base, n_base_charged, n_xpos, n_xneg;
    double energy;            /* retained energy: start energy + accepted changes (kT) */
    int64_t attempts[6];      /* trials per move id, auto-rejected ones included */
    int64_t accepts[6];
    uint32_t error_flags;     /* bit 0: cell capacity exceeded in binning;
                                 bit 1: capacity exceeded by an insertion;
                                 bit 2: (info) some neighbours of a domain did not fit
                                 on chip and were read from memory during its trials;
                                 bit 3: a domain did not fit its LDS pool and was
                                 skipped (an internal error; reported as CRMC_E_DEVICE) */
    int32_t n_cells;          /* cells per box edge */
    int32_t cell_capacity;
    int32_t max_cell_count;   /* most records any cell has held after re-binning */
    int64_t relocation_attempts; /* ion relocation trials (auto-rejected ones included) */
    int64_t relocation_accepts;
} crmc_obs;

/* Trial log record (56 bytes), written when logging is enabled. */
typedef struct {
    int64_t sweep, cell;        /* cell: first cell of the domain (linear index) */
    int32_t trial, replica;
    int32_t move, status;       /* status: 0 rejected, 1 accepted, 2 no participant */
    double dU, lnp, u;          /* dU in kT; lnp = log acceptance ratio; u uniform */
} crmc_trial_rec;

/*
 * Create a handle for n_replicas independent systems under the model of Sec.
 * II (screened Coulomb with lB, kappa and rc; excluded volume of Table I and
 * Table II; rho0 NA of the reference concentration of Sec. II C) and the
 * schedule fields of crmc_params.  No device work and no device memory;
 * returns CRMC_E_ARG for invalid params (rc <= 1.2, negative lB or eps,
 * trials outside 1..2^20, a workspace smaller than 256 bytes, ...).
 */
int crmc_create(const crmc_params* params, crmc_t* out);

/*
 * Caller-owned workspace.  crmc_workspace_size: after every replica is built,
 * *bytes = the device memory the handle's state needs at its current
 * settings: every replica's records, counts and observables, the plan and
 * tables of a sweep, the network with its Adam moments and the learned
 * proposal's work items (whether or not the proposal is on), and the per-cell
 * sums of crmc_energy.  Optional buffers come on top when enabled: the trial
 * log (56 bytes per record), the phase trace (48 bytes per record), training
 * rows (132 bytes per row), recorded features (128 bytes per particle of
 * every replica; included in the size once recording is on), and while
 * crmc_train, crmc_mlp_forward or crmc_mlp_gradient run, 4, 132 or 136
 * bytes per row, each buffer rounded up to 256 bytes.
 * crmc_set_workspace: hands over `bytes` of caller-owned device memory
 * (e.g. a torch uint8 tensor) before the first call that creates device
 * state (every call that reads or advances the replicas, sets the network
 * or enables a buffer); from then on every device buffer of the handle is
 * carved from it (first fit, 256-byte aligned, freed blocks reused) and a
 * request that does not fit fails with CRMC_E_NOMEM.  The caller keeps it
 * alive until crmc_destroy and must not touch it meanwhile.  Errors:
 * CRMC_E_STATE before all replicas are built (size) or once the handle has
 * device memory (attach); CRMC_E_ARG for NULL or fewer than 256 bytes.
 */
int crmc_workspace_size(crmc_t h, int64_t* bytes);
int crmc_set_workspace(crmc_t h, void* workspace, int64_t bytes);
/* Device memory of the handle now: the library's own live allocations and,
   with a workspace, its bytes in use and its largest free block (each
   pointer may be NULL).  Host only. */
int crmc_memory(crmc_t h, int64_t* own_bytes, int64_t* workspace_used, int64_t* workspace_largest_free);

/*
 * Define replica `replica` (Sec. II A: the system of fixed acid and base
 * groups, nanoparticle cores and free monovalent ions in a periodic box):
 * box edge L (periodic cube), n particles with
 * positions xyz (n*3 doubles, any real values; wrapped into the box), kind
 * (crmc_kind), optional charged flags (NULL = all sites neutral; ions are
 * always charged), optional group id per particle (NULL = 0) and n_cores
 * nanoparticle cores (core_xyz n_cores*3, radius core_R).  n_cells = 0 picks
 * the largest even count per edge whose cells are at least rc wide;
 * cell_capacity = 0 sizes the per-cell record capacity from the site density.
 * The initial order of particles is their stable binning into the unshifted
 * grid.  Returns CRMC_E_ARG when L < 4 rc, when n_cells is odd, below 4 or
 * gives cells narrower than rc, or when a cell already holds more than
 * cell_capacity particles; CRMC_E_STATE after the first sweep.  Host work
 * only: the replica's state goes to the device with the first call that
 * needs it.
 */
int crmc_build_cells(crmc_t h, int32_t replica, double L, int32_t n_cells, int32_t cell_capacity,
                     int32_t n, const double* xyz, const int32_t* kind, const int32_t* charged,
                     const int32_t* group, int32_t n_cores, const double* core_xyz,
                     const double* core_R);

/*
 * Run n_sweeps sweeps on every replica with the same conditions: pH, acid
 * pKa, combined-ion chemical potential mu_ion = pI_X+ = pI_X- (the input of
 * App. B; use crmc_pIX_from_salt for a salt pI_S), base pK and kappa from
 * crmc_params.  Asynchronous.
 */
int crmc_sweep(crmc_t h, double pH, double pKa, double mu_ion, int64_t n_sweeps);

/* Same with per-replica conditions (array of n_replicas). */
int crmc_sweep_ex(crmc_t h, const crmc_cond* per_replica, int64_t n_sweeps);

/*
 * crmc_sweep_ex with recovery from a cell running out of record capacity: the
 * sweeps run in chunks of `chunk`; the state after every good chunk is kept
 * on the host (as by crmc_export_state), and when a chunk ends with
 * CRMC_E_CAPACITY every replica's capacity is enlarged (by half, at least 32
 * records), the last good state is restored and the chunk is run again.
 * Capacity is storage only and the random numbers are counter based, so the
 * chain that results is the one an ample capacity gives.  *recoveries (may be
 * NULL) receives the number of enlargements.  Synchronizes after every chunk.
 * Errors: as crmc_sweep_ex; CRMC_E_CAPACITY after 16 enlargements;
 * CRMC_E_ARG when a grown cell no longer fits on-chip staging.
 */
int crmc_sweep_recover(crmc_t h, const crmc_cond* per_replica, int64_t n_sweeps, int64_t chunk,
                       int32_t* recoveries);

/*
 * Hybrid MD / CR-MC (Sec. III: blocks of MD steps between blocks of MC
 * steps): n_steps of Langevin molecular dynamics of the free ions of every
 * replica, velocity Verlet with time step dt and friction gamma (units sigma,
 * kT and the ion mass, tau = 1; the paper runs dt = 0.005 and n_MD = 400).
 * Sites and cores stay fixed.  Every ion starts the block with a
 * Maxwell-Boltzmann velocity; a step is v += dt/2 F; x += dt v (rounded to
 * the position lattice); F = F_c(x) - gamma v + sqrt(2 gamma / dt) xi;
 * v += dt/2 F, F_c = -grad E of the energy model (pair terms in the handle's
 * precision, summed in FP64; the cores' term in FP64; cells are at least
 * rc wide, so the 27 cells around an ion hold every partner).  After every
 * drift the ions are re-binned stably into the grid of the last sweep; the
 * random numbers of an ion come from Philox counters (step, cell, slot, 6)
 * (start velocity) and (step, cell, slot, 7) (noise), step the handle's
 * running count of MD steps (part of the exported state).  The retained energy
 * restarts from a from-scratch sum after the block.  Uses 72 bytes per record
 * slot of device memory (made at the first block, not in crmc_workspace_size).
 * Synchronizes.  Errors: CRMC_E_ARG for dt <= 0 or gamma < 0; CRMC_E_CAPACITY
 * when a cell overflowed.
 */
int crmc_md(crmc_t h, int64_t n_steps, double dt, double gamma);

/*
 * Counts, energy and move statistics of a replica (synchronizes): the
 * numbers of charged acid and base groups, whose means give the degree of
 * ionization alpha = <n_A->/n_A of Sec. III, the free-ion numbers, the
 * retained energy of Sec. II D (start energy plus accepted changes), and
 * attempts and acceptances per move of Sec. II C.  CRMC_E_CAPACITY when a cell
 * overflowed (the state is then not trustworthy), CRMC_E_STATE before build.
 */
int crmc_observe(crmc_t h, int32_t replica, crmc_obs* out);

/*
 * Per-sweep series [nA-, nB+, nX+, nX-] of a replica for sweeps
 * first .. first+count-1 (counted from build), written to out (count*4).
 * The library retains the last 16384 sweeps; sweeps outside that window (or
 * not yet run) return CRMC_E_ARG.
 */
int crmc_get_series(crmc_t h, int32_t replica, int64_t first, int64_t count, int32_t* out);

/*
 * Current particles of a replica in the library's order (cell order, then
 * order inside the cell): fixed-point positions xyz (cap*3), kind, charged,
 * site id (input index of the site; -1 for free ions).  *n_out = number of
 * particles; arrays are filled up to cap.
 */
int crmc_get_particles(crmc_t h, int32_t replica, int32_t cap, uint32_t* xyz, int32_t* kind,
                       int32_t* charged, int32_t* site_id, int32_t* n_out);

/* Total energy of the current state recomputed from scratch (kT). */
int crmc_energy(crmc_t h, int32_t replica, double* out);

/*
 * crmc_energy without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same kernel and the same summation
 * order as crmc_energy, so the result is bit-identical; its per-cell partial
 * sums and the replica descriptor go to a fixed device array of the library
 * (8 MiB + 1 KiB per GPU, held until the process ends), so replicas of at
 * most 2^20 cells are accepted (CRMC_E_ARG otherwise).  The replica's device
 * state must already exist (CRMC_E_STATE before the first call that creates
 * it, e.g. a sweep).  Calls on one GPU share that array: calls that overlap
 * in time on one GPU (other host threads, other handles) race and must be
 * serialized by the caller.  Synchronizes.
 */
int crmc_energy_noalloc(crmc_t h, int32_t replica, double* out);

/* Per-site count of sweeps at whose start the site was charged (n_sites values). */
int crmc_get_occupancy(crmc_t h, int32_t replica, int64_t cap, uint64_t* out, int64_t* n_out);

/* Histogram over sweeps of the number of ionized sites of each group g:
   out[off[g] + k], k = 0..n_sites(g); offsets written to off (n_groups+1). */
int crmc_get_group_hist(crmc_t h, int32_t replica, int64_t cap, int64_t* out, int32_t off_cap,
                        int32_t* off, int32_t* n_groups);

/*
 * Checkpoint and resume.  The state of a Markov chain is its particle
 * configuration (Sec. II: site charges, free-ion positions) plus what this
 * library accumulates along the chain; the random numbers are counter based,
 * so the sweep counter is all that is needed to continue the same chain.
 *
 * crmc_export_state writes, for every replica: the records of every cell in
 * their list order (ion picks depend on it), the running-energy terms, the
 * move counters, the per-site occupancy sums, the group histograms and the
 * retained series window; and the sweep counter, the proposal switch and, if
 * the network was ever used, its FP32 parameters with the Adam moments.  The
 * format is a versioned little-endian byte string of this library.  With
 * buf = NULL only *bytes = the size is written; a buffer smaller than *bytes
 * gives CRMC_E_ARG with *bytes set to the size needed.  Synchronizes.
 *
 * crmc_import_state restores such a state into a handle created with the same
 * n_replicas, precision and seed whose replicas were built from the same
 * inputs (same box, cell grid, sites, groups and cores; before its first sweep
 * or later); the cell capacity may differ as long as every cell's list fits.  A state that does not match, or is truncated or
 * malformed, gives CRMC_E_ARG and leaves the handle unchanged (the whole
 * state is checked on the host before any device memory is written); a
 * device or allocation error during the copy (CRMC_E_DEVICE, CRMC_E_NOMEM)
 * leaves the replicas in an undefined state.  Sweeping on
 * from the imported state with the same conditions continues the exported
 * chain bit for bit.  Conditions, logs, traces, timing and collected training
 * rows are not part of the state.  Synchronizes.
 */
int crmc_export_state(crmc_t h, void* buf, int64_t* bytes);
int crmc_import_state(crmc_t h, const void* buf, int64_t bytes);

/* Trial logging (testing): keep up to `capacity` records on the device. */
int crmc_enable_log(crmc_t h, int64_t capacity);
int crmc_read_log(crmc_t h, int64_t cap, crmc_trial_rec* out, int64_t* n_out);

/*
 * Learned site proposal (an extension of the method; the paper picks sites
 * uniformly, Sec. II C).  For an acid or base move the site is drawn with
 * probability q(i) = eps/m + (1 - eps) w_i / W over the m eligible sites of
 * the domain, w_i = p_i for a move that ionizes the site and 1 - p_i for one
 * that neutralizes it, W their sum; the acceptance uses ln q_rev - ln q_fwd in
 * place of the count ratio of the uniform pick (detailed balance, eq.
 * accrat).  p_i is the logistic of a 32 -> 128 -> 128 -> 1 ReLU network on
 * the site's environment: counts of charged particles within rc outside the
 * site's own cell, in 16 equal radial shells (exact integer thresholds
 * ceil((k rc / 16 / L 2^32)^2) on the squared lattice distance), the first 16
 * for charges opposite to the site's ionized charge, the last 16 for equal
 * ones.  Those cells are inactive during a colour phase, so the weights are
 * fixed during the domain's trials.  FP32 runs evaluate the network with BF16
 * matrix-core products (FP32 accumulation), FP64 runs in FP64.  The extra
 * random words of a trial come from Philox block 5 of its counter.
 *
 * crmc_set_proposal: learned = 1 turns it on with uniform weight eps in
 *   (0, 1] (eps = 1 is the uniform pick); learned = 0 off.
 * crmc_set_proposal_weights / crmc_get_proposal_weights: the network's
 *   CRMC_MLP_PARAMS FP32 parameters, W1[128][32], b1[128], W2[128][128],
 *   b2[128], w3[128], b3 (rows are output units); setting them restarts Adam.
 *   Before any are set they hold crmc_init_proposal_weights(h, seed ^
 *   0x5DEECE66D) of the handle's seed.
 * crmc_init_proposal_weights: He-uniform weights from a splitmix64 stream of
 *   seed: W1 and W2 uniform in +-sqrt(6 / fan_in), w3 in +-sqrt(3 / 128),
 *   biases zero; restarts Adam.  (With all weights zero the hidden units and
 *   their gradients vanish and training can move the output bias only.)
 * crmc_set_proposal_offsets: offsets added to the network's logit for the
 *   acid and the base sites of one replica (a calibration to the replica's
 *   conditions; any fixed offsets keep the chain exact).  Zero after
 *   crmc_build_cells; they take effect from the next sweep.
 * crmc_get_site_probabilities: p_i of every site of a replica as last
 *   evaluated (in its colour's phase of the latest sweep with the proposal
 *   on; 0 before any), indexed by particle input order; n >= the replica's
 *   particle count.
 * crmc_collect_training: while capacity > 0, every sweep appends one row per
 *   site and phase (32 features, then 1 if the site is ionized at the start
 *   of the phase) to a device buffer of that many rows (further rows are
 *   dropped); 0 stops and frees it.  crmc_training_rows / crmc_read_training
 *   read it back (rows of 33 floats).
 * crmc_train: epochs over the collected rows in shuffled minibatches of
 *   batch rows (seeded), mean binary cross-entropy, Adam (lr, betas 0.9 and
 *   0.999) on FP32 master parameters with BF16 matrix-core forward and
 *   backward products; last_loss receives the mean loss of the last epoch.
 * crmc_mlp_forward / crmc_mlp_gradient: the network's logits for n host
 *   feature rows (n x 32), and the mean-cross-entropy gradient and loss of n
 *   host rows (n x 33), on the same kernels (checks).
 * All synchronize; errors: CRMC_E_ARG for invalid arguments, CRMC_E_STATE
 * for training with fewer rows than one batch.
 */
#define CRMC_MLP_PARAMS 20865
int crmc_set_proposal(crmc_t h, int32_t learned, double eps);
int crmc_set_proposal_weights(crmc_t h, const float* w, int64_t n);
int crmc_get_proposal_weights(crmc_t h, float* w, int64_t n);
int crmc_init_proposal_weights(crmc_t h, uint64_t seed);
int crmc_set_proposal_offsets(crmc_t h, int32_t replica, double acid, double base);
int crmc_get_site_probabilities(crmc_t h, int32_t replica, double* out, int64_t n);
int crmc_collect_training(crmc_t h, int64_t capacity);
int crmc_training_rows(crmc_t h, int64_t* n);
int crmc_read_training(crmc_t h, int64_t first, int64_t count, float* out);
int crmc_train(crmc_t h, int32_t epochs, int32_t batch, double lr, uint64_t seed, double* last_loss);
int crmc_mlp_forward(crmc_t h, const float* X, int32_t n, float* logits);
/*
 * crmc_load_training: replaces the training rows with n host rows (n x 33,
 *   32 features then the 0/1 label) and stops collection; crmc_train then
 *   trains on them.  Synchronizes.  CRMC_E_ARG for n < 0 or NULL rows.
 * crmc_record_features: on = 1 keeps, per site, the 32 features the learned
 *   proposal's kernel evaluated in the site's colour phase of the latest
 *   sweep in which that kernel ran (proposal on, or rows being collected);
 *   crmc_get_site_features copies them (n >= 32 x the replica's particle
 *   count, row i for input particle i, zero for ions and before any
 *   evaluation).  A check of the features; it costs a store of 128 bytes per
 *   site and phase while on.  CRMC_E_STATE when recording is off.
 */
int crmc_load_training(crmc_t h, const float* rows, int64_t n);
int crmc_record_features(crmc_t h, int32_t on);
int crmc_get_site_features(crmc_t h, int32_t replica, float* out, int64_t n);
int crmc_mlp_gradient(crmc_t h, const float* rows, int32_t n, float* grad, double* loss);

/*
 * Launch-shape autotuner.  Times sweeps_per_candidate sweeps (after one
 * warm-up sweep) for every candidate pair of light_neighbours (which domains
 * run on one wavefront) and LDS pool size (lds_records) that the device and
 * the cell capacity allow, then keeps the fastest.  Neither knob changes any
 * result: the chain depends only on the seed, the schedule and the
 * conditions, so the tuning sweeps are ordinary sweeps of the chain (they
 * advance it by out->sweeps_used sweeps under per_replica conditions).
 * Every replica must be built.  Synchronizes.  A configuration tuned before
 * in the same process (same device, precision, schedule, proposal, seed,
 * and replicas of the same grids, capacities, cores, sites and built particle
 * counts) takes the cached shape without timing: out->reserved = 1,
 * n_candidates = 0 and sweeps_used = 0 (the chain does not advance).
 * Errors: CRMC_E_ARG for sweeps_per_candidate outside 1..100000,
 * CRMC_E_STATE before build; on a device error the previous launch shape is
 * kept.
 */
#define CRMC_TUNE_MAX 32
typedef struct {
    int32_t light_neighbours, lds_records; /* chosen launch shape */
    int32_t n_candidates;
    int32_t reserved;                      /* 1: the shape came from this process's cache */
    int64_t sweeps_used;                   /* sweeps the tuning advanced the chain by */
    double best_ms_per_sweep;
    double ms_per_sweep[CRMC_TUNE_MAX];    /* per candidate */
    int32_t cand_light[CRMC_TUNE_MAX], cand_lds[CRMC_TUNE_MAX];
} crmc_tune;
int crmc_autotune(crmc_t h, const crmc_cond* per_replica, int32_t sweeps_per_candidate, crmc_tune* out);

/*
 * Kernel timing.  While on, every kernel that crmc_sweep / crmc_sweep_ex
 * enqueues is bracketed by HIP events on the library's stream.
 * crmc_get_timing (synchronizes) returns the accumulated device milliseconds
 * and launch counts per kernel kind: [0] re-binning, planning and the learned
 * proposal's feature-and-network kernel, [1] trial phases,
 * [2] end-of-sweep bookkeeping; crmc_set_timing(h, 1) also resets them.
 */
int crmc_set_timing(crmc_t h, int32_t on);
int crmc_get_timing(crmc_t h, double ms[3], int64_t launches[3]);

/*
 * Per-workgroup trace of the trial-phase kernel (profiling): while capacity >
 * 0, every domain workgroup appends one record.  The clock is the device's
 * constant-rate wall clock (100 MHz on MI355X).
 */
typedef struct {
    uint64_t t0, t1;          /* wall clock at the start and end of the workgroup */
    uint32_t sweep, domain;   /* sweep; domain index over all replicas */
    int32_t colour, trials;   /* colour of the phase; trials the domain ran */
    int32_t neighbours, own;  /* neighbour records; records in the domain's cells */
    int32_t staged, hw_id;    /* neighbours held in LDS; compute unit that ran it */
} crmc_phase_trace;

int crmc_enable_trace(crmc_t h, int64_t capacity);
int crmc_read_trace(crmc_t h, int64_t cap, crmc_phase_trace* out, int64_t* n_out);

/* Philox4x32-10 on the device: n counter blocks (ctr n*4 words) with key
   (k0, k1) into out (n*4 words).  For checking the generator. */
int crmc_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out);

/* Combined-ion chemical potential from a symmetric salt (eq. pIXgen). */
double crmc_pIX_from_salt(double pIS, double pH, double pKw);

/*
 * Ungrouping (Sec. II D): the probability that a combined ion is one of its
 * subspecies is the ratio of their activities, 10^(pI_X - pI_i).  out[4] =
 * {S+ of X+, H+ of X+, S- of X-, OH- of X-} for salt potentials pIS_pos,
 * pIS_neg, the pH and pOH = pKw - pH, and the combined potentials pIX_pos,
 * pIX_neg the chain was run with; multiply by <n_X+> or <n_X-> for the
 * subspecies' means.  With pI_X from eq. pIXgen the salt ion and H+ (pH <=
 * pKw/2) or OH- (pH >= pKw/2) shares of one sign sum to 1; the rest of the
 * other sign is made of the ions that keep a non-neutral reservoir neutral.
 * Host only; CRMC_E_ARG for a NULL out or non-finite input.
 */
int crmc_ungroup_fractions(double pH, double pKw, double pIS_pos, double pIS_neg, double pIX_pos, double pIX_neg,
                           double* out);

/*
 * Ungrouping of the current state (Sec. II D): every free ion of the replica
 * is given the identity of one subspecies of its combined ion.  A cation is a
 * salt cation with probability frac[0] and H+ with probability frac[1], else
 * another ion of the reservoir; an anion is a salt anion with frac[2] and OH-
 * with frac[3] (frac as from crmc_ungroup_fractions; each pair sums to at most
 * 1).  Particle i in the library's order (that of crmc_get_particles) draws
 * u = unit53 of the first two Philox4x32-10 words of counter (draw low word,
 * draw high word, i, 5) under the replica's key; it is a salt ion if u <
 * frac_salt, H+ / OH- if u < frac_salt + frac_other, else another ion.
 * counts[6] = {S+, H+, other cations, S-, OH-, other anions}; labels (cap
 * entries, may be NULL with cap = 0) get per particle 0 (not a free ion), 1
 * (salt ion), 2 (H+ or OH-) or 3 (other); *n_out = particle count.  Different
 * draw values give independent ungroupings of the same state.  Synchronizes;
 * CRMC_E_ARG for fractions outside [0, 1] or summing to more than 1 per sign.
 */
int crmc_ungroup(crmc_t h, int32_t replica, const double frac[4], uint64_t draw, int64_t counts[6],
                 int8_t* labels, int64_t cap, int64_t* n_out);

const char* crmc_last_error(crmc_t h);
void crmc_destroy(crmc_t h);

#ifdef __cplusplus
}
#endif

#endif /* CRMC_H */
