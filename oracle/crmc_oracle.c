/*
 * Plain FP64 CPU oracle for charge-regulation Monte Carlo (CR-MC).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU baseline
 * of the benchmark can compare the GPU path against a slow, obviously correct
 * implementation.  It shares no code with the GPU path.
 *
 * What it implements (Curk, Yuan, Luijten, "Accelerated simulation method for
 * charge regulation effects"):
 *   - the three grouped reactions A <-> A- + X+, B <-> B+ + X-, 0 <-> X+ + X-
 *     (Sec. II B, eqs. acid_new, base_new, salt_new);
 *   - the six moves (forward and reverse of each reaction), proposed with equal
 *     probability, participants chosen uniformly, auto-reject when no eligible
 *     participant exists (Sec. II C);
 *   - the Metropolis acceptance probabilities of Sec. II C (eqs. acidacc,
 *     MCmetro, the acid/base reverse and forward forms, MCsaltf, MCmetro2),
 *     written in the log10 parametrisation pH, pOH, pK, pI_X (Sec. II C);
 *   - energy changes computed from the changed particles only, keeping the old
 *     energy between moves (Sec. II D).
 *
 * Two schedules:
 *   paper mode  - one global move at a time, insertion uniform in the whole box
 *                 (the literal algorithm of Sec. II C);
 *   cell mode   - the same moves restricted to one cell of a randomly shifted
 *                 cubic grid; cells of one parity class ("colour") are mutually
 *                 non-interacting (cell width >= cutoff) and are processed one
 *                 after another; the grid shift is redrawn every sweep so that
 *                 cells overlap across sweeps.  The acceptance is the paper's
 *                 formula with V replaced by the cell volume and every count
 *                 replaced by the cell's count (detailed balance, eq. accrat,
 *                 with a proposal density uniform in the cell).  This is the
 *                 schedule the GPU path runs, word for word.
 *
 * Energy model (screened Coulomb + excluded volume, positions fixed):
 *   E = sum_{i<j, r<rc} lB q_i q_j exp(-kappa r)/r
 *     + sum_{pairs with at least one free ion, r<2^(1/6)} 4 eps (r^-12 - r^-6) + eps
 *     + sum_{ion, core} expanded WCA with Delta = R - 1/2     (Table II, eq. LJe)
 * Site-site excluded volume and bonds are constant (sites never move) and are
 * left out.  The Coulomb cutoff is decided exactly on the integer squared
 * distance of the fixed-point coordinates.  A free-ion pair closer than 0.5
 * (or an ion closer than Delta + 0.5 to a core centre) has infinite energy.
 *
 * Learned proposal (cell mode, optional; not in the paper): the site of an
 * acid/base move is drawn with probability q(i) = eps/m + (1-eps) w_i / W over
 * the m eligible sites of the domain, w_i = p_i for a move that ionizes and
 * 1 - p_i for one that neutralizes, where p_i is the output of a small
 * multilayer perceptron (32 -> 128 -> 128 -> 1, ReLU, logistic) on the site's
 * environment: counts of charged particles in 16 equal radial shells within
 * rc, split into charges opposite to and equal to the site's ionized charge,
 * over the particles that lie outside the site's own cell.  Those cells are
 * inactive for the whole colour phase, so p_i is fixed during the domain's
 * trials and the Metropolis-Hastings ratio q_rev / q_fwd (replacing the
 * uniform-pick count ratio of Sec. II C) makes every trial satisfy detailed
 * balance for the frozen environment.
 *
 * Ion relocation trials (cell mode, optional, off by default; not in the
 * paper, whose ions move by molecular dynamics between MC blocks): after the
 * reaction trials of a domain, a free ion picked uniformly is removed and
 * re-inserted at a point drawn like an insertion of its sign, accepted with
 * min(1, (V_new / V_old) exp(-dU)) (eq. accrat for that proposal).
 *
 * Test aids that change no arithmetic: a trial limit stops a run after its
 * first n trials in processing order; a state can be loaded in a given
 * particle order at a given sweep index (to continue a chain that another
 * program ran); the grid of the current sweep can be binned without running
 * trials (to read site features); a domain filter runs only chosen domains of
 * the first colour phase of a sweep.
 *
 * Pinned by the tests: closed forms (ideal ions, salt-only box, high-salt
 * limit), the exact enumeration of a 12-site ring, the one-site quadrature,
 * brute-force energy differences on every trial, the two schedules against
 * each other, and a fixed-grid negative control.
 *
 * Everything is FP64.  Random numbers are Philox4x32-10 (Salmon, Moraes, Dror,
 * Shaw, SC'11), written here from its published definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ACID 1
#define ORC_BASE 2
#define ORC_XPOS 3
#define ORC_XNEG 4
#define ORC_NEUTRAL 5

#define TAG_TRIAL 1u
#define TAG_SHIFT 2u
#define TAG_PAPER 3u
#define TAG_PAIR 4u
#define TAG_UNGROUP 5u
#define TAG_MDVEL 6u
#define TAG_MDNOISE 7u

static const double LN10 = 2.302585092994045684017991454684364208;
static const double TWO32 = 4294967296.0;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                              */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Data                                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t x[3];
    int32_t kind;
    int32_t charged; /* sites: 0/1; free ions: always 1 */
    int32_t sid;     /* site index in input order; -1 for free ions */
    double v[3];     /* velocity during a molecular-dynamics block (free ions) */
} orc_particle;

typedef struct {
    int64_t sweep, cell, trial; /* cell = -1 in paper mode; trial = global index there */
    int32_t move;               /* 0..5; auto-rejected trials keep their move id */
    int32_t status;             /* 0 rejected, 1 accepted, 2 auto-rejected (no participant) */
    double dU;                  /* beta * Delta E (NaN when auto-rejected) */
    double lnp;                 /* log acceptance ratio (NaN when auto-rejected) */
    double u;                   /* uniform in [0,1) used for the decision */
} orc_trial;

typedef struct {
    int n, cap;
    orc_particle* p;
} orc_list;

typedef struct {
    /* parameters */
    double L, lB, kappa, rc, eps, rho0NA;
    int ion_coupling;
    uint64_t R2; /* exact integer Coulomb cutoff on squared lattice distance */
    uint32_t key[2];
    /* conditions */
    double lnKA, lnKB, lnKion;
    /* cell schedule */
    int n;           /* cells per dimension */
    int trials;      /* trials per active cell per phase */
    int fixed_grid;  /* 1 = never shift the grid (test-only negative control) */
    int pairing;     /* 1 = trials act on reflection-paired cells, 0 = single cells */
    int site_trials; /* extra trials per 16 ionizable sites of a domain */
    int ion_trials;  /* ion relocation trials per cell of a domain, after the reaction trials */
    /* state, in global order */
    int np, npcap;
    orc_particle* P;
    int nc;
    uint32_t* core_x; /* nc*3 */
    double* core_delta;
    uint64_t sweep;
    int64_t paper_trial;
    uint64_t md_step; /* molecular-dynamics steps run so far (counter of their random numbers) */
    double E; /* running energy: brute force at build, then += accepted dU */
    int64_t attempts[6], accepts[6];
    int64_t reloc_att, reloc_acc; /* ion relocation trials */
    /* cell lists during a sweep */
    orc_list* cells;
    int ncells;
    orc_particle* flat; /* scratch: all particles in one array */
    int flat_cap;
    /* logging */
    orc_trial* log;
    int64_t log_cap, log_n;
    /* checking: when set, every trial's local dU is compared with a brute-force
       energy difference and the largest deviation is kept */
    int check_dU;
    double max_dU_err;
    /* test aid: when trial_limit >= 0, trials beyond the first trial_limit
       (counted from the last orc_set_trial_limit, in processing order) are
       skipped; they are not logged and change nothing */
    int64_t trial_limit, trials_run;
    /* test aid: when dom_filter_n >= 0, a sweep runs only the domains of its
       first colour phase whose first cell is listed (every domain of one
       colour is independent of the others, so their trials are exactly those
       of the full sweep) and skips the other seven phases */
    int dom_filter_n;
    int32_t* dom_filter;
    /* learned proposal */
    int learned;
    double lp_eps;
    double lp_off[2];    /* logit offsets of acid and base sites */
    double* lp_par;      /* ORC_MLP_PARAMS values */
    double* lp_phat;     /* per site id: network output for the current phase */
    int lp_nsites;
    uint64_t R2sh[17];   /* shell k holds lattice squared distances in [R2sh[k], R2sh[k+1]) */
} orc_sys;

/* network parameters: W1[128][32], b1[128], W2[128][128], b2[128], w3[128], b3 */
#define ORC_MLP_IN 32
#define ORC_MLP_H 128
#define ORC_MLP_PARAMS (ORC_MLP_H * ORC_MLP_IN + ORC_MLP_H + ORC_MLP_H * ORC_MLP_H + ORC_MLP_H + ORC_MLP_H + 1)
#define ORC_P_B1 (ORC_MLP_H * ORC_MLP_IN)
#define ORC_P_W2 (ORC_P_B1 + ORC_MLP_H)
#define ORC_P_B2 (ORC_P_W2 + ORC_MLP_H * ORC_MLP_H)
#define ORC_P_W3 (ORC_P_B2 + ORC_MLP_H)
#define ORC_P_B3 (ORC_P_W3 + ORC_MLP_H)

/* ------------------------------------------------------------------------- */
/* Small helpers                                                              */
/* ------------------------------------------------------------------------- */
static int charge_of(int kind, int charged)
{
    if (kind == ORC_ACID) return charged ? -1 : 0;
    if (kind == ORC_BASE) return charged ? 1 : 0;
    if (kind == ORC_XPOS) return 1;
    if (kind == ORC_XNEG) return -1;
    return 0;
}
static int is_ion(int kind) { return kind == ORC_XPOS || kind == ORC_XNEG; }

/* floor(w * m / 2^32): uniform integer in [0, m) from one 32-bit word */
static uint32_t pick32(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w * m) >> 32); }

/* floor((hi*2^32 + lo) * m / 2^64): uniform integer in [0, m) from two words */
static uint32_t pick64(uint32_t hi, uint32_t lo, uint32_t m)
{
    uint64_t low = ((uint64_t)lo * m) >> 32;
    uint64_t top = (uint64_t)hi * m + low;
    return (uint32_t)(top >> 32);
}

/* uniform double in [0,1) with 53 random bits */
static double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

uint64_t orc_cutoff_R2(double rc, double L)
{
    double t = (rc / L) * TWO32;
    return (uint64_t)ceil(t * t);
}

/* x in [any real] -> fixed point on the periodic lattice of 2^32 points per box edge */
void orc_to_fixed(int64_t n3, const double* xyz, double L, uint32_t* out)
{
    for (int64_t i = 0; i < n3; ++i) {
        double f = xyz[i] / L;
        f -= floor(f);
        double v = floor(f * TWO32);
        if (v >= TWO32) v = 0.0;
        out[i] = (uint32_t)v;
    }
}

/* cell boundaries b_k = ceil(k 2^32 / n); cell of relative coordinate y */
static uint64_t cell_lo(int k, int n) { return (((uint64_t)k << 32) + (uint64_t)n - 1) / (uint64_t)n; }
static int cell_of(uint32_t y, int n) { return (int)(((uint64_t)y * (uint64_t)n) >> 32); }

/* ------------------------------------------------------------------------- */
/* Energies                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t x[3];
    int q;       /* charge in this state */
    int ion;     /* 1 if a free ion */
    int present; /* 0 if absent in this state */
} orc_state_pt;

static void lattice_delta(const uint32_t* a, const uint32_t* b, int32_t d[3])
{
    for (int k = 0; k < 3; ++k) d[k] = (int32_t)(b[k] - a[k]);
}

static double wca(double r2, double eps)
{
    if (r2 < 0.25) return INFINITY;
    double ir2 = 1.0 / r2;
    double ir6 = ir2 * ir2 * ir2;
    return 4.0 * eps * (ir6 * ir6 - ir6) + eps;
}

/* energy of one pair; either member may be absent */
static double pair_energy(const orc_sys* S, const orc_state_pt* a, const orc_state_pt* b)
{
    if (!a->present || !b->present) return 0.0;
    if (!S->ion_coupling && (a->ion || b->ion)) return 0.0;
    int32_t d[3];
    lattice_delta(a->x, b->x, d);
    uint64_t r2i = (uint64_t)((int64_t)d[0] * d[0]) + (uint64_t)((int64_t)d[1] * d[1]) +
                   (uint64_t)((int64_t)d[2] * d[2]);
    double s = S->L / TWO32;
    double r2 = (double)r2i * s * s;
    double e = 0.0;
    if (S->eps > 0.0 && (a->ion || b->ion) && r2 < 1.2599210498948731647672106) /* 2^(1/3) */
        e += wca(r2, S->eps);
    if (r2i < S->R2 && a->q != 0 && b->q != 0) {
        double r = sqrt(r2);
        e += S->lB * (double)(a->q * b->q) * exp(-S->kappa * r) / r;
    }
    return e;
}

/* energy of a free ion with all nanoparticle cores (expanded WCA, Table II) */
static double core_energy(const orc_sys* S, const orc_state_pt* a)
{
    if (!a->present || !a->ion || !S->ion_coupling || S->eps <= 0.0) return 0.0;
    double e = 0.0;
    double s = S->L / TWO32;
    for (int c = 0; c < S->nc; ++c) {
        int32_t d[3];
        lattice_delta(a->x, &S->core_x[3 * c], d);
        double dx = d[0] * s, dy = d[1] * s, dz = d[2] * s;
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double sh = r - S->core_delta[c];
        /* the expanded potential is defined outside the core only (r > Delta);
           closer than Delta + 1/2 (inside included) is an overlap */
        if (sh < 0.5) return INFINITY;
        if (sh < 1.122462048309373) /* 2^(1/6) */
            e += wca(sh * sh, S->eps);
    }
    return e;
}

static orc_state_pt as_state(const orc_particle* p)
{
    orc_state_pt s;
    memcpy(s.x, p->x, sizeof s.x);
    s.q = charge_of(p->kind, p->charged);
    s.ion = is_ion(p->kind);
    s.present = 1;
    return s;
}

static int total_count(const orc_sys* S, int in_cells)
{
    if (!in_cells) return S->np;
    int t = 0;
    for (int c = 0; c < S->ncells; ++c) t += S->cells[c].n;
    return t;
}

/* brute-force total energy: every pair once, plus ion-core terms */
static double energy_of_array(const orc_sys* S, const orc_particle* P, int np)
{
    double E = 0.0;
    for (int i = 0; i < np; ++i) {
        orc_state_pt a = as_state(&P[i]);
        E += core_energy(S, &a);
        for (int j = i + 1; j < np; ++j) {
            orc_state_pt b = as_state(&P[j]);
            E += pair_energy(S, &a, &b);
        }
    }
    return E;
}

double orc_energy(const orc_sys* S) { return energy_of_array(S, S->P, S->np); }

/* ------------------------------------------------------------------------- */
/* Creation and set-up                                                        */
/* ------------------------------------------------------------------------- */
orc_sys* orc_create(double L, int n_cells, double lB, double kappa, double rc, double eps,
                    double rho0NA, int ion_coupling, uint64_t seed, uint32_t replica)
{
    orc_sys* S = (orc_sys*)calloc(1, sizeof(orc_sys));
    S->L = L; S->n = n_cells; S->lB = lB; S->kappa = kappa; S->rc = rc; S->eps = eps;
    S->rho0NA = rho0NA; S->ion_coupling = ion_coupling;
    S->R2 = orc_cutoff_R2(rc, L);
    S->key[0] = (uint32_t)seed;
    S->key[1] = (uint32_t)(seed >> 32) ^ replica;
    S->trials = 1;
    S->trial_limit = -1;
    S->dom_filter_n = -1;
    S->ncells = n_cells * n_cells * n_cells;
    S->cells = (orc_list*)calloc((size_t)S->ncells, sizeof(orc_list));
    return S;
}

void orc_destroy(orc_sys* S)
{
    if (!S) return;
    for (int c = 0; c < S->ncells; ++c) free(S->cells[c].p);
    free(S->cells); free(S->flat); free(S->P); free(S->core_x); free(S->core_delta);
    free(S->dom_filter);
    free(S->lp_par); free(S->lp_phat);
    free(S);
}

/* ------------------------------------------------------------------------- */
/* Learned proposal: features and network                                     */
/* ------------------------------------------------------------------------- */
int orc_mlp_params(void) { return ORC_MLP_PARAMS; }

/* logit of the network for one feature vector */
double orc_mlp_logit(const double* par, const double* x)
{
    double h1[ORC_MLP_H], h2[ORC_MLP_H];
    for (int o = 0; o < ORC_MLP_H; ++o) {
        double a = par[ORC_P_B1 + o];
        for (int i = 0; i < ORC_MLP_IN; ++i) a += par[o * ORC_MLP_IN + i] * x[i];
        h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < ORC_MLP_H; ++o) {
        double a = par[ORC_P_B2 + o];
        for (int i = 0; i < ORC_MLP_H; ++i) a += par[ORC_P_W2 + o * ORC_MLP_H + i] * h1[i];
        h2[o] = a > 0.0 ? a : 0.0;
    }
    double z = par[ORC_P_B3];
    for (int i = 0; i < ORC_MLP_H; ++i) z += par[ORC_P_W3 + i] * h2[i];
    return z;
}

/* site probability used by the proposal: the logistic of the logit, kept
   inside [1e-6, 1 - 1e-6] so that every eligible site has positive weight */
static double site_prob(double z)
{
    double p = 1.0 / (1.0 + exp(-z));
    if (p < 1e-6) p = 1e-6;
    if (p > 1.0 - 1e-6) p = 1.0 - 1e-6;
    return p;
}

/* Mean binary cross-entropy of the network over n labelled feature vectors
   and its gradient with respect to every parameter (backpropagation). */
double orc_mlp_loss_grad(const double* par, const double* X, const double* y, int n, double* grad)
{
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * ORC_MLP_PARAMS);
    for (int r = 0; r < n; ++r) {
        const double* x = X + (size_t)r * ORC_MLP_IN;
        double a1[ORC_MLP_H], h1[ORC_MLP_H], a2[ORC_MLP_H], h2[ORC_MLP_H];
        for (int o = 0; o < ORC_MLP_H; ++o) {
            double a = par[ORC_P_B1 + o];
            for (int i = 0; i < ORC_MLP_IN; ++i) a += par[o * ORC_MLP_IN + i] * x[i];
            a1[o] = a;
            h1[o] = a > 0.0 ? a : 0.0;
        }
        for (int o = 0; o < ORC_MLP_H; ++o) {
            double a = par[ORC_P_B2 + o];
            for (int i = 0; i < ORC_MLP_H; ++i) a += par[ORC_P_W2 + o * ORC_MLP_H + i] * h1[i];
            a2[o] = a;
            h2[o] = a > 0.0 ? a : 0.0;
        }
        double z = par[ORC_P_B3];
        for (int i = 0; i < ORC_MLP_H; ++i) z += par[ORC_P_W3 + i] * h2[i];
        /* BCE with logits: softplus(z) - y z, stable form */
        loss += (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y[r] * z;
        if (!grad) continue;
        const double dz = (1.0 / (1.0 + exp(-z)) - y[r]) / n;
        double d2[ORC_MLP_H], d1[ORC_MLP_H];
        grad[ORC_P_B3] += dz;
        for (int i = 0; i < ORC_MLP_H; ++i) {
            grad[ORC_P_W3 + i] += dz * h2[i];
            d2[i] = a2[i] > 0.0 ? dz * par[ORC_P_W3 + i] : 0.0;
        }
        for (int i = 0; i < ORC_MLP_H; ++i) d1[i] = 0.0;
        for (int o = 0; o < ORC_MLP_H; ++o) {
            if (d2[o] == 0.0) continue;
            grad[ORC_P_B2 + o] += d2[o];
            for (int i = 0; i < ORC_MLP_H; ++i) {
                grad[ORC_P_W2 + o * ORC_MLP_H + i] += d2[o] * h1[i];
                d1[i] += d2[o] * par[ORC_P_W2 + o * ORC_MLP_H + i];
            }
        }
        for (int o = 0; o < ORC_MLP_H; ++o) {
            const double g = a1[o] > 0.0 ? d1[o] : 0.0;
            if (g == 0.0) continue;
            grad[ORC_P_B1 + o] += g;
            for (int i = 0; i < ORC_MLP_IN; ++i) grad[o * ORC_MLP_IN + i] += g * x[i];
        }
    }
    return loss / n;
}

/* one Adam step (Kingma & Ba 2015) on every parameter; m, v are the moment
   estimates, t the 1-based step number */
void orc_adam_step(double* par, const double* grad, double* m, double* v, int64_t t, double lr, double b1,
                   double b2, double eps)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int i = 0; i < ORC_MLP_PARAMS; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        par[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* shell of a lattice squared distance below the cutoff: the largest k with
   R2sh[k] <= d2 (R2sh[0] = 0, R2sh[16] = the cutoff) */
static int shell_of(const orc_sys* S, uint64_t d2)
{
    int k = 15;
    while (k > 0 && d2 < S->R2sh[k]) --k;
    return k;
}

/* Features of site p in cell c: charged particles of the 26 neighbour cells
   within rc, by shell; x[0..15] charges opposite to the site's ionized
   charge, x[16..31] equal ones. */
static void site_features(const orc_sys* S, const orc_particle* p, int c, double* x)
{
    int n = S->n;
    int cx = c % n, cy = (c / n) % n, cz = c / (n * n);
    int qion = p->kind == ORC_ACID ? -1 : 1;
    for (int i = 0; i < ORC_MLP_IN; ++i) x[i] = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                int nc = ((cx + dx + n) % n) + n * (((cy + dy + n) % n) + n * ((cz + dz + n) % n));
                const orc_list* l = &S->cells[nc];
                for (int j = 0; j < l->n; ++j) {
                    int q = charge_of(l->p[j].kind, l->p[j].charged);
                    if (q == 0) continue;
                    int32_t d[3];
                    lattice_delta(p->x, l->p[j].x, d);
                    uint64_t d2 = (uint64_t)((int64_t)d[0] * d[0]) + (uint64_t)((int64_t)d[1] * d[1]) +
                                  (uint64_t)((int64_t)d[2] * d[2]);
                    if (d2 >= S->R2) continue;
                    x[(q * qion < 0 ? 0 : 16) + shell_of(S, d2)] += 1.0;
                }
            }
}

/* features of every site in the cell grid of the current sweep (tests) */
int orc_features_of_cell_sites(const orc_sys* S, int c, int cap, int32_t* sid, double* X)
{
    const orc_list* l = &S->cells[c];
    int k = 0;
    for (int j = 0; j < l->n; ++j) {
        const orc_particle* p = &l->p[j];
        if (p->kind != ORC_ACID && p->kind != ORC_BASE) continue;
        if (k < cap) {
            sid[k] = p->sid;
            site_features(S, p, c, X + (size_t)k * ORC_MLP_IN);
        }
        ++k;
    }
    return k;
}

/* Enable the learned proposal with the given network parameters and uniform
   mixing eps (0 < eps <= 1; eps = 1 is the plain uniform proposal). */
/* Offsets added to the network's logit of acid and base sites (a fixed
   per-condition calibration; any fixed weights keep the chain exact). */
void orc_set_learned_offsets(orc_sys* S, double acid, double base)
{
    S->lp_off[0] = acid;
    S->lp_off[1] = base;
}

int orc_set_learned(orc_sys* S, const double* par, double eps, int on)
{
    if (on && (!(eps > 0.0) || eps > 1.0)) return -1;
    S->learned = on;
    S->lp_eps = eps;
    if (!S->lp_par) S->lp_par = (double*)malloc(sizeof(double) * ORC_MLP_PARAMS);
    if (par) memcpy(S->lp_par, par, sizeof(double) * ORC_MLP_PARAMS);
    for (int k = 0; k <= 16; ++k) {
        double t = (k * S->rc / 16.0 / S->L) * TWO32;
        S->R2sh[k] = (uint64_t)ceil(t * t);
    }
    S->R2sh[0] = 0;
    return 0;
}

void orc_set_conditions(orc_sys* S, double pH, double pKa, double pKb, double pIXp, double pIXm,
                        double pKw)
{
    double pOH = pKw - pH;
    S->lnKA = (pH - pKa - pIXp) * LN10;
    S->lnKB = (pOH - pKb - pIXm) * LN10;
    S->lnKion = -(pIXp + pIXm) * LN10;
}

void orc_set_kappa(orc_sys* S, double kappa) { S->kappa = kappa; }

void orc_set_schedule(orc_sys* S, int trials_per_cell, int fixed_grid, int pairing, int site_trials)
{
    S->trials = trials_per_cell;
    S->fixed_grid = fixed_grid;
    S->pairing = pairing;
    S->site_trials = site_trials;
}

void orc_set_log(orc_sys* S, orc_trial* log, int64_t cap)
{
    S->log = log; S->log_cap = cap; S->log_n = 0;
}
int64_t orc_log_count(const orc_sys* S) { return S->log_n; }

void orc_set_ion_trials(orc_sys* S, int ion_trials) { S->ion_trials = ion_trials; }
void orc_relocation_stats(const orc_sys* S, int64_t out[2]) { out[0] = S->reloc_att; out[1] = S->reloc_acc; }
void orc_set_check(orc_sys* S, int on) { S->check_dU = on; S->max_dU_err = 0.0; }
void orc_set_trial_limit(orc_sys* S, int64_t n) { S->trial_limit = n; S->trials_run = 0; }
double orc_max_dU_err(const orc_sys* S) { return S->max_dU_err; }

static void ensure_cap(orc_sys* S, int need)
{
    if (need <= S->npcap) return;
    int c = S->npcap ? S->npcap : 64;
    while (c < need) c *= 2;
    S->P = (orc_particle*)realloc(S->P, (size_t)c * sizeof(orc_particle));
    S->npcap = c;
}

static void list_push(orc_list* l, const orc_particle* p)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 16;
        l->p = (orc_particle*)realloc(l->p, (size_t)l->cap * sizeof(orc_particle));
    }
    l->p[l->n++] = *p;
}

/* stable binning of the global array into the cells of grid shift o */
static void bin_into_cells(orc_sys* S, const uint32_t o[3])
{
    int n = S->n;
    for (int c = 0; c < S->ncells; ++c) S->cells[c].n = 0;
    for (int i = 0; i < S->np; ++i) {
        const orc_particle* p = &S->P[i];
        int cx = cell_of(p->x[0] - o[0], n), cy = cell_of(p->x[1] - o[1], n), cz = cell_of(p->x[2] - o[2], n);
        list_push(&S->cells[cx + n * (cy + n * cz)], p);
    }
}

/* concatenate the cell lists back into the global array (cell index order) */
static void gather_from_cells(orc_sys* S)
{
    int np = total_count(S, 1);
    ensure_cap(S, np);
    int k = 0;
    for (int c = 0; c < S->ncells; ++c)
        for (int j = 0; j < S->cells[c].n; ++j) S->P[k++] = S->cells[c].p[j];
    S->np = k;
}

/* Particles in input order; the build then puts them into the cells of the
   unshifted grid (stable) and takes that as the initial global order. */
int orc_set_particles(orc_sys* S, int np, const uint32_t* xyz, const int32_t* kind,
                      const int32_t* charged, const int32_t* sid)
{
    ensure_cap(S, np > 0 ? np : 1);
    S->np = np;
    for (int i = 0; i < np; ++i) {
        orc_particle* p = &S->P[i];
        p->x[0] = xyz[3 * i]; p->x[1] = xyz[3 * i + 1]; p->x[2] = xyz[3 * i + 2];
        p->kind = kind[i];
        p->charged = is_ion(kind[i]) ? 1 : (charged ? charged[i] : 0);
        p->sid = sid ? sid[i] : (is_ion(kind[i]) ? -1 : i);
    }
    int maxsid = -1;
    for (int i = 0; i < np; ++i)
        if (S->P[i].sid > maxsid) maxsid = S->P[i].sid;
    free(S->lp_phat);
    S->lp_nsites = maxsid + 1;
    S->lp_phat = (double*)calloc((size_t)(maxsid + 2), sizeof(double));
    uint32_t o[3] = {0, 0, 0};
    bin_into_cells(S, o);
    gather_from_cells(S);
    S->E = orc_energy(S);
    S->sweep = 0;
    S->paper_trial = 0;
    memset(S->attempts, 0, sizeof S->attempts);
    memset(S->accepts, 0, sizeof S->accepts);
    return 0;
}

/* Test aid: the state of a chain that another program ran, at the start of
   sweep `sweep`: particles in the given order, which becomes the global order
   the next sweep's stable binning starts from (the order a sweep leaves is
   cell order of its grid, then list order inside each cell).  The running
   energy restarts from a brute-force sum (or from NaN when with_energy is 0:
   that sum is quadratic in the particle count, and the local energy changes
   do not need it) and the move counters from zero.  Nothing else changes: the random numbers are counter based, so the next
   sweep draws exactly the words the other program's sweep drew. */
int orc_load_state(orc_sys* S, int np, const uint32_t* xyz, const int32_t* kind, const int32_t* charged,
                   const int32_t* sid, uint64_t sweep, int with_energy)
{
    ensure_cap(S, np > 0 ? np : 1);
    S->np = np;
    int maxsid = -1;
    for (int i = 0; i < np; ++i) {
        orc_particle* p = &S->P[i];
        p->x[0] = xyz[3 * i]; p->x[1] = xyz[3 * i + 1]; p->x[2] = xyz[3 * i + 2];
        p->kind = kind[i];
        p->charged = is_ion(kind[i]) ? 1 : charged[i];
        p->sid = is_ion(kind[i]) ? -1 : sid[i];
        if (p->sid > maxsid) maxsid = p->sid;
    }
    if (maxsid + 1 > S->lp_nsites || !S->lp_phat) {
        free(S->lp_phat);
        S->lp_nsites = maxsid + 1;
        S->lp_phat = (double*)calloc((size_t)(maxsid + 2), sizeof(double));
    }
    S->E = with_energy ? orc_energy(S) : NAN;
    S->sweep = sweep;
    S->paper_trial = 0;
    S->reloc_att = S->reloc_acc = 0;
    memset(S->attempts, 0, sizeof S->attempts);
    memset(S->accepts, 0, sizeof S->accepts);
    return 0;
}

int orc_set_cores(orc_sys* S, int nc, const uint32_t* xyz, const double* radius)
{
    free(S->core_x); free(S->core_delta);
    S->nc = nc;
    S->core_x = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (size_t)(nc > 0 ? nc : 1));
    S->core_delta = (double*)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    for (int c = 0; c < nc; ++c) {
        memcpy(&S->core_x[3 * c], &xyz[3 * c], 3 * sizeof(uint32_t));
        S->core_delta[c] = radius[c] - 0.5; /* Delta = R - r with ion radius r = sigma/2 */
    }
    S->E = orc_energy(S);
    return 0;
}

int orc_num_particles(const orc_sys* S) { return S->np; }

int orc_get_particles(const orc_sys* S, int cap, uint32_t* xyz, int32_t* kind, int32_t* charged,
                      int32_t* sid)
{
    int n = S->np < cap ? S->np : cap;
    for (int i = 0; i < n; ++i) {
        const orc_particle* p = &S->P[i];
        xyz[3 * i] = p->x[0]; xyz[3 * i + 1] = p->x[1]; xyz[3 * i + 2] = p->x[2];
        kind[i] = p->kind; charged[i] = p->charged; sid[i] = p->sid;
    }
    return S->np;
}

/* counts: [nA, nA-, nB, nB+, nX+, nX-] */
void orc_counts(const orc_sys* S, int64_t out[6])
{
    memset(out, 0, 6 * sizeof(int64_t));
    for (int i = 0; i < S->np; ++i) {
        const orc_particle* p = &S->P[i];
        if (p->kind == ORC_ACID) { out[0]++; out[1] += p->charged; }
        else if (p->kind == ORC_BASE) { out[2]++; out[3] += p->charged; }
        else if (p->kind == ORC_XPOS) out[4]++;
        else if (p->kind == ORC_XNEG) out[5]++;
    }
}

double orc_running_energy(const orc_sys* S) { return S->E; }
uint64_t orc_sweep_index(const orc_sys* S) { return S->sweep; }
void orc_move_stats(const orc_sys* S, int64_t att[6], int64_t acc[6])
{
    memcpy(att, S->attempts, sizeof S->attempts);
    memcpy(acc, S->accepts, sizeof S->accepts);
}

/* ------------------------------------------------------------------------- */
/* One trial, shared by both schedules                                        */
/* ------------------------------------------------------------------------- */
/* A "changed" particle: an existing one (index into the particle set being
   moved on, old state from there) or a new one (old state absent). */
typedef struct {
    int idx;           /* index into the working set; -1 for an inserted ion */
    orc_state_pt old_s, new_s;
} orc_change;

/* dU = E(new) - E(old), restricted to the terms that involve changed particles:
   changed-vs-unchanged pairs, the pair between the changed particles, and
   ion-core terms. 'set' holds every particle of the system (np of them). */
static double local_dU(const orc_sys* S, const orc_particle* set, int np, const orc_change* ch, int nch)
{
    double dU = 0.0;
    for (int a = 0; a < nch; ++a) {
        dU += core_energy(S, &ch[a].new_s) - core_energy(S, &ch[a].old_s);
        for (int j = 0; j < np; ++j) {
            int skip = 0;
            for (int b = 0; b < nch; ++b)
                if (ch[b].idx == j) skip = 1;
            if (skip) continue;
            orc_state_pt pj = as_state(&set[j]);
            double en = pair_energy(S, &ch[a].new_s, &pj);
            double eo = pair_energy(S, &ch[a].old_s, &pj);
            dU += en - eo;
        }
    }
    if (nch == 2)
        dU += pair_energy(S, &ch[0].new_s, &ch[1].new_s) - pair_energy(S, &ch[0].old_s, &ch[1].old_s);
    return dU;
}

/* A trial acts on a "domain": one cell, two mutually non-interacting cells of
   the same colour (cell mode), or the whole box (paper mode).  Its particles
   are the concatenation of the domain's lists; picks are uniform over the
   domain's eligible particles in that order. */
typedef struct {
    int ncell;                  /* number of cells (1 or 2); 1 in paper mode */
    orc_list* list[2];
    int cell[2];                /* linear cell index (cell mode) */
    uint32_t ins_base[2][3];    /* insertion region per cell: lattice origin */
    uint32_t ins_width[2][3];   /* lattice width; 0 = whole box (paper mode) */
    double lnZ[2];              /* ln(rho0 NA / q) where q is the insertion density
                                   of a point in that cell: 1/(ncell V_cell) */
    int nreact;
    int react[3];
    int paper;
    const orc_sys* sys; /* learned proposal: weights by site id (NULL: uniform picks) */
} orc_dom;

/* domain-order index -> (cell j, local index) */
static void dom_locate(const orc_dom* D, int g, int* j, int* i)
{
    if (D->ncell == 2 && g >= D->list[0]->n) { *j = 1; *i = g - D->list[0]->n; }
    else { *j = 0; *i = g; }
}

static int dom_size(const orc_dom* D)
{
    int n = 0;
    for (int j = 0; j < D->ncell; ++j) n += D->list[j]->n;
    return n;
}

static orc_particle* dom_at(const orc_dom* D, int g)
{
    int j, i;
    dom_locate(D, g, &j, &i);
    return &D->list[j]->p[i];
}

/* domain-order index of the k-th particle satisfying the predicate */
static int kth(const orc_dom* D, int kind, int charged, int k)
{
    int n = dom_size(D);
    for (int g = 0; g < n; ++g) {
        const orc_particle* p = dom_at(D, g);
        if (p->kind == kind && (is_ion(kind) || p->charged == charged)) {
            if (k == 0) return g;
            --k;
        }
    }
    return -1;
}

static int count_of(const orc_dom* D, int kind, int charged)
{
    int c = 0, n = dom_size(D);
    for (int g = 0; g < n; ++g) {
        const orc_particle* p = dom_at(D, g);
        if (p->kind == kind && (is_ion(kind) || p->charged == charged)) ++c;
    }
    return c;
}

/* weight of a site for a move that ionizes (fwd = 1) or neutralizes it */
static double site_weight(const orc_dom* D, const orc_particle* p, int fwd)
{
    double ph = D->sys->lp_phat[p->sid];
    return fwd ? ph : 1.0 - ph;
}

/* sum of the weights of the eligible sites of a class */
static double class_weight(const orc_dom* D, int kind, int charged, int fwd)
{
    double w = 0.0;
    int n = dom_size(D);
    for (int g = 0; g < n; ++g) {
        const orc_particle* p = dom_at(D, g);
        if (p->kind == kind && p->charged == charged) w += site_weight(D, p, fwd);
    }
    return w;
}

/* the learned pick: uniform over the m eligible sites with probability eps
   (words: e, then k as in the plain pick), otherwise proportional to the
   weights (a 53-bit uniform t scaled by the total weight W, the first
   eligible site whose cumulative weight exceeds it; the last one if
   rounding leaves none) */
static int learned_pick(const orc_dom* D, int kind, int charged, int fwd, int m, double W, uint32_t we,
                        uint32_t wk, uint32_t wt0, uint32_t wt1)
{
    double eps = D->sys->lp_eps;
    if ((double)we * (1.0 / TWO32) < eps) return kth(D, kind, charged, (int)pick32(wk, (uint32_t)m));
    double target = unit53(wt0, wt1) * W, cum = 0.0;
    int n = dom_size(D), last = -1;
    for (int g = 0; g < n; ++g) {
        const orc_particle* p = dom_at(D, g);
        if (p->kind != kind || p->charged != charged) continue;
        cum += site_weight(D, p, fwd);
        last = g;
        if (cum > target) return g;
    }
    return last;
}

/* log of the learned proposal probability of site p among m eligible sites of
   total weight W */
static double ln_q(const orc_dom* D, const orc_particle* p, int fwd, int m, double W)
{
    double eps = D->sys->lp_eps;
    return log(eps / m + (1.0 - eps) * site_weight(D, p, fwd) / W);
}

/* insertion point: choose a cell of the domain uniformly (word wc), then a
   lattice point uniformly inside it (two words per coordinate, ws[0..5]);
   paper mode: one word per coordinate over the whole box */
static int insertion_point(const orc_dom* D, uint32_t wc, const uint32_t* ws, uint32_t out[3])
{
    int j = D->ncell == 1 ? 0 : (int)pick32(wc, (uint32_t)D->ncell);
    for (int d = 0; d < 3; ++d) {
        if (D->ins_width[j][d] == 0)
            out[d] = ws[2 * d];
        else
            out[d] = D->ins_base[j][d] + pick64(ws[2 * d], ws[2 * d + 1], D->ins_width[j][d]);
    }
    return j;
}

/* Every particle of the system in one array, for the energy sums; base[j]
   is the offset of domain cell j inside it. */
static orc_particle* flatten(orc_sys* S, const orc_dom* D, int* nall, int base[2])
{
    if (D->paper) {
        *nall = D->list[0]->n; base[0] = 0;
        return D->list[0]->p;
    }
    int n = total_count(S, 1);
    if (n > S->flat_cap) {
        S->flat_cap = n + 64;
        S->flat = (orc_particle*)realloc(S->flat, (size_t)S->flat_cap * sizeof(orc_particle));
    }
    int k = 0;
    for (int c = 0; c < S->ncells; ++c) {
        for (int j = 0; j < D->ncell; ++j)
            if (c == D->cell[j]) base[j] = k;
        for (int i = 0; i < S->cells[c].n; ++i) S->flat[k++] = S->cells[c].p[i];
    }
    *nall = k;
    return S->flat;
}

static void swap_remove(orc_list* l, int i)
{
    l->p[i] = l->p[l->n - 1];
    l->n--;
}

/* One trial of a domain.  reloc = 0: one of the six moves of Sec. II C.
   reloc = 1: an ion relocation (move id 6, not one of the paper's moves; it
   stands in for the motion the paper's ions get from molecular dynamics): a
   free ion of the domain picked uniformly is removed and re-inserted at a
   point drawn like an insertion of its sign.  The proposal is symmetric up to
   the insertion densities, so ln p = ln V_new - ln V_old - dU (eq. accrat). */
static void do_trial(orc_sys* S, orc_dom* D, const uint32_t* w, int64_t cell, int64_t trial, int reloc)
{
    uint32_t k = pick32(w[0], (uint32_t)(2 * D->nreact));
    int reaction = D->react[k >> 1];
    int dir = (int)(k & 1u);
    int move = reloc ? 6 : 2 * reaction + dir;

    int m0a = count_of(D, ORC_ACID, 0), mca = count_of(D, ORC_ACID, 1);
    int m0b = count_of(D, ORC_BASE, 0), mcb = count_of(D, ORC_BASE, 1);
    int npos = count_of(D, ORC_XPOS, 1), nneg = count_of(D, ORC_XNEG, 1);

    int auto_reject = 0;
    int site = -1, del_pos = -1, del_neg = -1, ins_pos = 0, ins_neg = 0;
    double lnp_counts = 0.0; /* every term of ln p except the volume terms and -dU */
    switch (move) {
    case 0: /* acid forward: A -> A-, X+ in */
        if (m0a == 0) { auto_reject = 1; break; }
        site = kth(D, ORC_ACID, 0, (int)pick32(w[1], (uint32_t)m0a));
        ins_pos = 1;
        lnp_counts = log((double)m0a) - log((double)(mca + 1)) - log((double)(npos + 1)) + S->lnKA;
        break;
    case 1: /* acid reverse: A- -> A, X+ out */
        if (mca == 0 || npos == 0) { auto_reject = 1; break; }
        site = kth(D, ORC_ACID, 1, (int)pick32(w[1], (uint32_t)mca));
        del_pos = kth(D, ORC_XPOS, 1, (int)pick32(w[2], (uint32_t)npos));
        lnp_counts = log((double)mca) + log((double)npos) - log((double)(m0a + 1)) - S->lnKA;
        break;
    case 2: /* base forward: B -> B+, X- in */
        if (m0b == 0) { auto_reject = 1; break; }
        site = kth(D, ORC_BASE, 0, (int)pick32(w[1], (uint32_t)m0b));
        ins_neg = 1;
        lnp_counts = log((double)m0b) - log((double)(mcb + 1)) - log((double)(nneg + 1)) + S->lnKB;
        break;
    case 3: /* base reverse: B+ -> B, X- out */
        if (mcb == 0 || nneg == 0) { auto_reject = 1; break; }
        site = kth(D, ORC_BASE, 1, (int)pick32(w[1], (uint32_t)mcb));
        del_neg = kth(D, ORC_XNEG, 1, (int)pick32(w[3], (uint32_t)nneg));
        lnp_counts = log((double)mcb) + log((double)nneg) - log((double)(m0b + 1)) - S->lnKB;
        break;
    case 4: /* salt pair in */
        ins_pos = ins_neg = 1;
        lnp_counts = -log((double)(npos + 1)) - log((double)(nneg + 1)) + S->lnKion;
        break;
    case 5: /* salt pair out */
        if (npos == 0 || nneg == 0) { auto_reject = 1; break; }
        del_pos = kth(D, ORC_XPOS, 1, (int)pick32(w[2], (uint32_t)npos));
        del_neg = kth(D, ORC_XNEG, 1, (int)pick32(w[3], (uint32_t)nneg));
        lnp_counts = log((double)npos) + log((double)nneg) - S->lnKion;
        break;
    case 6: { /* ion relocation: the k-th ion, cations first */
        if (npos + nneg == 0) { auto_reject = 1; break; }
        const int kk = (int)pick32(w[1], (uint32_t)(npos + nneg));
        if (kk < npos) { del_pos = kth(D, ORC_XPOS, 1, kk); ins_pos = 1; }
        else { del_neg = kth(D, ORC_XNEG, 1, kk - npos); ins_neg = 1; }
        break;
    }
    }
    if (D->sys && move <= 3 && !auto_reject) {
        /* learned site pick: the count ratio of the uniform picks becomes
           ln q_rev(i | s') - ln q_fwd(i | s) */
        const int kind = move <= 1 ? ORC_ACID : ORC_BASE, fwd = !(move & 1), ch = move & 1;
        const int m = kind == ORC_ACID ? (ch ? mca : m0a) : (ch ? mcb : m0b);
        const int mr = (kind == ORC_ACID ? (ch ? m0a : mca) : (ch ? m0b : mcb)) + 1;
        const double W = class_weight(D, kind, ch, fwd);
        site = learned_pick(D, kind, ch, fwd, m, W, w[20], w[1], w[21], w[22]);
        const orc_particle* ps = dom_at(D, site);
        const double Wr = class_weight(D, kind, !ch, !fwd) + site_weight(D, ps, !fwd);
        const double lnq = ln_q(D, ps, !fwd, mr, Wr) - ln_q(D, ps, fwd, m, W);
        switch (move) {
        case 0: lnp_counts = lnq - log((double)(npos + 1)) + S->lnKA; break;
        case 1: lnp_counts = lnq + log((double)npos) - S->lnKA; break;
        case 2: lnp_counts = lnq - log((double)(nneg + 1)) + S->lnKB; break;
        default: lnp_counts = lnq + log((double)nneg) - S->lnKB; break;
        }
    }
    if (move == 6) S->reloc_att++; else S->attempts[move]++;
    double u = unit53(w[16], w[17]);
    if (auto_reject) {
        if (S->log && S->log_n < S->log_cap) {
            orc_trial* t = &S->log[S->log_n++];
            t->sweep = (int64_t)S->sweep; t->cell = cell; t->trial = trial; t->move = move;
            t->status = 2; t->dU = NAN; t->lnp = NAN; t->u = u;
        }
        return;
    }

    /* positions of inserted ions, and the volume terms: each inserted ion
       contributes +ln(rho0 NA / q), each deleted one -ln(rho0 NA / q), with q
       the density at which the reverse move would propose its position */
    uint32_t xp[3], xn[3];
    int jp = -1, jn = -1;
    double lnvol = 0.0;
    if (ins_pos) { jp = insertion_point(D, w[18], &w[4], xp); lnvol += D->lnZ[jp]; }
    if (ins_neg) { jn = insertion_point(D, w[19], &w[10], xn); lnvol += D->lnZ[jn]; }
    int sj = -1, si = -1, pj = -1, pi = -1, nj = -1, ni = -1;
    if (site >= 0) dom_locate(D, site, &sj, &si);
    if (del_pos >= 0) { dom_locate(D, del_pos, &pj, &pi); lnvol -= D->lnZ[pj]; }
    if (del_neg >= 0) { dom_locate(D, del_neg, &nj, &ni); lnvol -= D->lnZ[nj]; }

    int base[2] = {0, 0}, nall = 0;
    orc_particle* all = flatten(S, D, &nall, base);

    orc_change ch[2];
    int nch = 0;
    if (site >= 0) {
        orc_change* c = &ch[nch++];
        const orc_particle* p = &D->list[sj]->p[si];
        c->idx = base[sj] + si;
        c->old_s = as_state(p);
        c->new_s = c->old_s;
        c->new_s.q = charge_of(p->kind, !p->charged);
    }
    if (del_pos >= 0) {
        orc_change* c = &ch[nch++];
        c->idx = base[pj] + pi;
        c->old_s = as_state(&D->list[pj]->p[pi]);
        c->new_s = c->old_s; c->new_s.present = 0;
    }
    if (del_neg >= 0) {
        orc_change* c = &ch[nch++];
        c->idx = base[nj] + ni;
        c->old_s = as_state(&D->list[nj]->p[ni]);
        c->new_s = c->old_s; c->new_s.present = 0;
    }
    if (ins_pos) {
        orc_change* c = &ch[nch++];
        c->idx = -1;
        memcpy(c->new_s.x, xp, sizeof xp);
        c->new_s.q = 1; c->new_s.ion = 1; c->new_s.present = 1;
        c->old_s = c->new_s; c->old_s.present = 0;
    }
    if (ins_neg) {
        orc_change* c = &ch[nch++];
        c->idx = -1;
        memcpy(c->new_s.x, xn, sizeof xn);
        c->new_s.q = -1; c->new_s.ion = 1; c->new_s.present = 1;
        c->old_s = c->new_s; c->old_s.present = 0;
    }

    double dU = local_dU(S, all, nall, ch, nch);
    double lnp = lnp_counts + lnvol - dU;
    int accept = u < exp(lnp < 0.0 ? lnp : 0.0);

    if (S->check_dU && isfinite(dU)) {
        /* brute force: total energy of the new state minus that of the old */
        double e_old = energy_of_array(S, all, nall);
        orc_particle* tmp = (orc_particle*)malloc((size_t)(nall + 2) * sizeof(orc_particle));
        int m = 0;
        for (int j = 0; j < nall; ++j) {
            int gone = 0;
            for (int b = 0; b < nch; ++b)
                if (ch[b].idx == j && !ch[b].new_s.present) gone = 1;
            if (gone) continue;
            tmp[m] = all[j];
            if (site >= 0 && j == base[sj] + si) tmp[m].charged = !tmp[m].charged;
            ++m;
        }
        if (ins_pos) { memcpy(tmp[m].x, xp, sizeof xp); tmp[m].kind = ORC_XPOS; tmp[m].charged = 1; tmp[m].sid = -1; ++m; }
        if (ins_neg) { memcpy(tmp[m].x, xn, sizeof xn); tmp[m].kind = ORC_XNEG; tmp[m].charged = 1; tmp[m].sid = -1; ++m; }
        double e_new = energy_of_array(S, tmp, m);
        free(tmp);
        double err = fabs((e_new - e_old) - dU) / (fabs(dU) > 1.0 ? fabs(dU) : 1.0);
        if (err > S->max_dU_err) S->max_dU_err = err;
    }

    if (S->log && S->log_n < S->log_cap) {
        orc_trial* t = &S->log[S->log_n++];
        t->sweep = (int64_t)S->sweep; t->cell = cell; t->trial = trial; t->move = move;
        t->status = accept; t->dU = dU; t->lnp = lnp; t->u = u;
    }
    if (!accept) return;

    /* commit: flip in place; deletions, each by moving the last element of its
       cell into the hole (when both deleted ions sit in one cell, the one at
       the higher index goes first); insertions appended to their cells, X+
       before X- */
    if (move == 6) S->reloc_acc++; else S->accepts[move]++;
    S->E += dU;
    if (site >= 0) D->list[sj]->p[si].charged = !D->list[sj]->p[si].charged;
    if (del_pos >= 0 && del_neg >= 0 && pj == nj && ni > pi) {
        swap_remove(D->list[nj], ni);
        swap_remove(D->list[pj], pi);
    } else {
        if (del_pos >= 0) swap_remove(D->list[pj], pi);
        if (del_neg >= 0) swap_remove(D->list[nj], ni);
    }
    orc_particle q;
    q.charged = 1; q.sid = -1;
    if (ins_pos) { memcpy(q.x, xp, sizeof xp); q.kind = ORC_XPOS; list_push(D->list[jp], &q); }
    if (ins_neg) { memcpy(q.x, xn, sizeof xn); q.kind = ORC_XNEG; list_push(D->list[jn], &q); }
}

/* ------------------------------------------------------------------------- */
/* Cell schedule                                                              */
/* ------------------------------------------------------------------------- */
void orc_shift(const orc_sys* S, uint64_t sweep, uint32_t o[3])
{
    if (S->fixed_grid) { o[0] = o[1] = o[2] = 0; return; }
    uint32_t ctr[4] = {(uint32_t)sweep, 0u, 0u, TAG_SHIFT}, w[4];
    orc_philox(ctr, S->key, w);
    o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
}

/* Partner of active cell a (of M active cells of one colour) in a phase: the
   reflection a -> (c - a) mod M about a point c drawn from the phase's own
   counter.  It pairs far-apart cells, is an involution, and has no fixed
   point when M is even (one when M is odd). */
uint32_t orc_partner(const orc_sys* S, uint64_t sweep, int colour, uint32_t a, uint32_t M)
{
    uint32_t ctr[4] = {(uint32_t)sweep, (uint32_t)colour, 0u, TAG_PAIR}, w[4];
    orc_philox(ctr, S->key, w);
    uint32_t r = pick32(w[0], M);
    uint64_t c = ((uint64_t)M - 1u + 2ull * M - 2ull * r) % M; /* (M - 1 - 2r) mod M */
    return (uint32_t)((c + M - a) % M);
}

static void trial_words(const orc_sys* S, uint32_t tag, uint32_t c0, uint32_t c1, uint32_t c2base, uint32_t w[24])
{
    for (uint32_t b = 0; b < 6; ++b) {
        uint32_t ctr[4] = {c0, c1, c2base + b, tag};
        orc_philox(ctr, S->key, &w[4 * b]);
    }
}

static void set_cell_region(const orc_sys* S, orc_dom* D, int j, int c, const uint32_t o[3], double lnZ0)
{
    int n = S->n;
    int cc[3] = {c % n, (c / n) % n, c / (n * n)};
    double lnV = 0.0;
    for (int d = 0; d < 3; ++d) {
        uint64_t lo = cell_lo(cc[d], n), hi = cell_lo(cc[d] + 1, n);
        D->ins_base[j][d] = o[d] + (uint32_t)lo;
        D->ins_width[j][d] = (uint32_t)(hi - lo);
        lnV += log((double)(hi - lo));
    }
    D->lnZ[j] = lnZ0 + lnV;
    D->list[j] = &S->cells[c];
    D->cell[j] = c;
}

/* Test aid: bin the particles into the shifted grid of the current sweep
   (the first step of a sweep) without running trials or advancing, so that
   orc_features_of_cell_sites reads the cells the sweep's first phase sees. */
void orc_prepare_sweep(orc_sys* S)
{
    uint32_t o[3];
    orc_shift(S, S->sweep, o);
    bin_into_cells(S, o);
}

/* Test aid: n >= 0 restricts the next sweeps to the listed domains (by their
   first cell) of the first colour phase; n < 0 turns the filter off. */
void orc_set_domain_filter(orc_sys* S, int n, const int32_t* first_cells)
{
    free(S->dom_filter);
    S->dom_filter = NULL;
    S->dom_filter_n = n;
    if (n > 0) {
        S->dom_filter = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        memcpy(S->dom_filter, first_cells, sizeof(int32_t) * (size_t)n);
    }
}

static int domain_selected(const orc_sys* S, int colour, int first_cell)
{
    if (S->dom_filter_n < 0) return 1;
    if (colour != 0) return 0;
    for (int i = 0; i < S->dom_filter_n; ++i)
        if (S->dom_filter[i] == first_cell) return 1;
    return 0;
}

static void one_sweep(orc_sys* S, int32_t* series)
{
    int n = S->n, h = n / 2;
    uint32_t M = (uint32_t)(h * h * h);
    uint32_t o[3];
    orc_shift(S, S->sweep, o);
    bin_into_cells(S, o);
    double lnZ0 = log(S->rho0NA) + 3.0 * log(S->L / TWO32);
    for (int colour = 0; colour < 8; ++colour) {
        int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
        for (uint32_t a = 0; a < M; ++a) {
            uint32_t b = S->pairing ? orc_partner(S, S->sweep, colour, a, M) : a;
            if (b < a) continue; /* the domain is handled from its lower member */
            uint32_t mem[2] = {a, b};
            orc_dom D;
            memset(&D, 0, sizeof D);
            D.ncell = (b == a) ? 1 : 2;
            double lnk = log((double)D.ncell);
            for (int j = 0; j < D.ncell; ++j) {
                uint32_t m = mem[j];
                int i = (int)(m % (uint32_t)h), jj = (int)((m / (uint32_t)h) % (uint32_t)h), kk = (int)(m / (uint32_t)(h * h));
                int c = (2 * i + px) + n * ((2 * jj + py) + n * (2 * kk + pz));
                set_cell_region(S, &D, j, c, o, lnZ0 + lnk);
            }
            if (!domain_selected(S, colour, D.cell[0])) continue;
            /* static move set and trial count: the domain's site content does
               not depend on the state */
            int has_acid = 0, has_base = 0, nsites = 0;
            for (int j = 0; j < D.ncell; ++j)
                for (int q = 0; q < D.list[j]->n; ++q) {
                    if (D.list[j]->p[q].kind == ORC_ACID) { has_acid = 1; ++nsites; }
                    if (D.list[j]->p[q].kind == ORC_BASE) { has_base = 1; ++nsites; }
                }
            D.nreact = 0;
            if (has_acid) D.react[D.nreact++] = 0;
            if (has_base) D.react[D.nreact++] = 1;
            D.react[D.nreact++] = 2;
            if (S->learned) {
                /* the domain's site probabilities: their environment (the
                   neighbour cells) does not change during this phase */
                D.sys = S;
                for (int j = 0; j < D.ncell; ++j)
                    for (int q = 0; q < D.list[j]->n; ++q) {
                        const orc_particle* sp = &D.list[j]->p[q];
                        if (sp->kind != ORC_ACID && sp->kind != ORC_BASE) continue;
                        double x[ORC_MLP_IN];
                        site_features(S, sp, D.cell[j], x);
                        S->lp_phat[sp->sid] =
                            site_prob(orc_mlp_logit(S->lp_par, x) + S->lp_off[sp->kind == ORC_ACID ? 0 : 1]);
                    }
            }
            /* the reaction trials, then the ion relocation trials */
            int ntr_react = S->trials * D.ncell + (nsites * S->site_trials + 15) / 16;
            int ntr = ntr_react + S->ion_trials * D.ncell;
            for (int t = 0; t < ntr; ++t) {
                if (S->trial_limit >= 0 && S->trials_run >= S->trial_limit) break;
                S->trials_run++;
                uint32_t w[24];
                trial_words(S, TAG_TRIAL, (uint32_t)S->sweep, (uint32_t)D.cell[0], (uint32_t)t * 8u, w);
                do_trial(S, &D, w, D.cell[0], t, t >= ntr_react);
            }
        }
    }
    gather_from_cells(S);
    if (series) {
        int64_t cnt[6];
        orc_counts(S, cnt);
        series[0] = (int32_t)cnt[1]; series[1] = (int32_t)cnt[3];
        series[2] = (int32_t)cnt[4]; series[3] = (int32_t)cnt[5];
    }
    S->sweep++;
}

/* series: nsweeps x [nA-, nB+, nX+, nX-] after each sweep (may be NULL) */
int orc_sweeps(orc_sys* S, int64_t nsweeps, int32_t* series)
{
    for (int64_t s = 0; s < nsweeps; ++s) one_sweep(S, series ? &series[4 * s] : NULL);
    return 0;
}

/* Ungrouping (Sec. II D): every free ion of the current state, in global
   order, is given the identity of one subspecies of its combined ion.  A
   cation is a salt cation with probability frac[0] and H+ with probability
   frac[1] (each 10^(pI_X+ - pI_i)), otherwise another ion of the reservoir;
   an anion is a salt anion with frac[2], OH- with frac[3].  The uniform of
   particle i is unit53 of the first two Philox words of counter
   (draw low word, draw high word, i, tag 5).  labels[i]: 0 not a free ion,
   1 salt ion, 2 H+ or OH-, 3 other; counts: salt cations, H+, other cations,
   salt anions, OH-, other anions. */
void orc_ungroup(const orc_sys* S, const double frac[4], uint64_t draw, int64_t counts[6], int32_t* labels)
{
    memset(counts, 0, 6 * sizeof(int64_t));
    for (int i = 0; i < S->np; ++i) {
        const orc_particle* p = &S->P[i];
        if (!is_ion(p->kind)) {
            if (labels) labels[i] = 0;
            continue;
        }
        uint32_t ctr[4] = {(uint32_t)draw, (uint32_t)(draw >> 32), (uint32_t)i, TAG_UNGROUP}, w[4];
        orc_philox(ctr, S->key, w);
        const double u = unit53(w[0], w[1]);
        const int neg = p->kind == ORC_XNEG;
        const double fs = frac[2 * neg], fo = frac[2 * neg + 1];
        const int lab = u < fs ? 1 : (u < fs + fo ? 2 : 3);
        counts[3 * neg + lab - 1]++;
        if (labels) labels[i] = lab;
    }
}

/* ------------------------------------------------------------------------- */
/* Hybrid MD / CR-MC: Langevin dynamics of the free ions between sweeps       */
/* ------------------------------------------------------------------------- */
/* Force on free ion a from the rest of the system: -grad of the energy E of
   the energy model (screened Coulomb inside the exact integer cutoff, the
   excluded volume of every pair with a free ion, the expanded excluded volume
   of the cores).  Brute force over every other particle. */
static void ion_force(const orc_sys* S, const orc_particle* P, int np, int a, double f[3])
{
    const double s = S->L / TWO32;
    f[0] = f[1] = f[2] = 0.0;
    const orc_particle* pa = &P[a];
    const int qa = charge_of(pa->kind, pa->charged);
    for (int j = 0; j < np; ++j) {
        if (j == a) continue;
        const orc_particle* pb = &P[j];
        if (!S->ion_coupling) continue; /* ideal ions feel nothing */
        int32_t d[3];
        lattice_delta(pb->x, pa->x, d); /* from b to a */
        const uint64_t r2i = (uint64_t)((int64_t)d[0] * d[0]) + (uint64_t)((int64_t)d[1] * d[1]) +
                             (uint64_t)((int64_t)d[2] * d[2]);
        const double dx = d[0] * s, dy = d[1] * s, dz = d[2] * s;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double g = 0.0; /* -dU/dr / r */
        const int qb = charge_of(pb->kind, pb->charged);
        if (r2i < S->R2 && qa != 0 && qb != 0) {
            const double r = sqrt(r2);
            g += S->lB * (double)(qa * qb) * exp(-S->kappa * r) * (1.0 + S->kappa * r) / (r2 * r);
        }
        if (S->eps > 0.0 && r2 < 1.2599210498948731647672106) {
            const double ir2 = 1.0 / r2, ir6 = ir2 * ir2 * ir2;
            g += 4.0 * S->eps * (12.0 * ir6 * ir6 - 6.0 * ir6) * ir2;
        }
        f[0] += g * dx; f[1] += g * dy; f[2] += g * dz;
    }
    if (S->ion_coupling && S->eps > 0.0) {
        for (int c = 0; c < S->nc; ++c) {
            int32_t d[3];
            lattice_delta(&S->core_x[3 * c], pa->x, d);
            const double dx = d[0] * s, dy = d[1] * s, dz = d[2] * s;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double sh = r - S->core_delta[c];
            if (sh < 1.122462048309373) {
                const double ir = 1.0 / sh, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
                const double g = 4.0 * S->eps * (12.0 * ir6 * ir6 - 6.0 * ir6) * ir / r;
                f[0] += g * dx; f[1] += g * dy; f[2] += g * dz;
            }
        }
    }
}

/* three standard normal deviates (Box-Muller) from one Philox block */
static void normals3(const orc_sys* S, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double z[3])
{
    uint32_t ctr[4] = {c0, c1, c2, tag}, w[4];
    orc_philox(ctr, S->key, w);
    const double TWO_PI = 6.283185307179586476925286766559;
    const double u1 = ((double)w[0] + 1.0) / TWO32, u2 = (double)w[1] / TWO32;
    const double u3 = ((double)w[2] + 1.0) / TWO32, u4 = (double)w[3] / TWO32;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    z[0] = r1 * cos(TWO_PI * u2);
    z[1] = r1 * sin(TWO_PI * u2);
    z[2] = r2 * cos(TWO_PI * u4);
}

/* Forces of all free ions (zero for other particles) in global order (tests). */
void orc_forces(const orc_sys* S, double* F)
{
    for (int i = 0; i < S->np; ++i) {
        if (is_ion(S->P[i].kind)) ion_force(S, S->P, S->np, i, &F[3 * i]);
        else F[3 * i] = F[3 * i + 1] = F[3 * i + 2] = 0.0;
    }
}

/* A molecular-dynamics block: nsteps velocity-Verlet steps of length dt for
   the free ions with a Langevin thermostat of friction gamma (the hybrid
   MD/MC protocol of Sec. III, units sigma, kT and the ion mass, so tau = 1).
   Sites and cores stay where they are.  At the start every ion gets a
   Maxwell-Boltzmann velocity; one step is
     v += dt/2 F;  x += dt v (rounded to the lattice);  F = F_c(x) - gamma v
     + sqrt(2 gamma / dt) xi;  v += dt/2 F,
   with F = F_c at the start.  The ions stay binned in the grid of the last
   sweep: after every drift they are re-binned into it stably, and the
   random numbers of an ion are addressed by its cell and slot there:
   Philox counter (step, cell, slot, 6) for the initial velocity and
   (step, cell, slot, 7) for the noise of a step, step the running count of
   MD steps.  The retained energy restarts from a brute-force sum.  Returns
   the mean of v^2 per component over the ions and the steps (the
   thermostat's temperature check). */
double orc_md(orc_sys* S, int64_t nsteps, double dt, double gamma)
{
    uint32_t o[3] = {0u, 0u, 0u};
    if (S->sweep > 0) orc_shift(S, S->sweep - 1, o);
    bin_into_cells(S, o);
    const double to_lat = TWO32 / S->L;
    const double noise = sqrt(2.0 * gamma / dt);
    double v2sum = 0.0;
    int64_t v2n = 0;
    /* initial velocities and forces, in the current binning */
    gather_from_cells(S);
    double* F = (double*)calloc((size_t)3 * (size_t)(S->np > 0 ? S->np : 1), sizeof(double));
    {
        int k = 0;
        for (int c = 0; c < S->ncells; ++c)
            for (int j = 0; j < S->cells[c].n; ++j, ++k) {
                orc_particle* p = &S->P[k];
                if (!is_ion(p->kind)) { p->v[0] = p->v[1] = p->v[2] = 0.0; continue; }
                normals3(S, (uint32_t)S->md_step, (uint32_t)c, (uint32_t)j, TAG_MDVEL, p->v);
            }
        for (int i = 0; i < S->np; ++i)
            if (is_ion(S->P[i].kind)) ion_force(S, S->P, S->np, i, &F[3 * i]);
    }
    for (int64_t st = 0; st < nsteps; ++st) {
        const uint64_t g = S->md_step + (uint64_t)st;
        for (int i = 0; i < S->np; ++i) {
            orc_particle* p = &S->P[i];
            if (!is_ion(p->kind)) continue;
            for (int k = 0; k < 3; ++k) {
                p->v[k] += 0.5 * dt * F[3 * i + k];
                p->x[k] = (uint32_t)((int64_t)p->x[k] + llround(dt * p->v[k] * to_lat));
            }
        }
        /* re-bin (stable) into the same grid; forces travel with nothing: they are recomputed */
        bin_into_cells(S, o);
        gather_from_cells(S);
        int k = 0;
        for (int c = 0; c < S->ncells; ++c)
            for (int j = 0; j < S->cells[c].n; ++j, ++k) {
                orc_particle* p = &S->P[k];
                if (!is_ion(p->kind)) continue;
                double fc[3], z[3];
                ion_force(S, S->P, S->np, k, fc);
                normals3(S, (uint32_t)g, (uint32_t)c, (uint32_t)j, TAG_MDNOISE, z);
                for (int q = 0; q < 3; ++q) {
                    F[3 * k + q] = fc[q] - gamma * p->v[q] + noise * z[q];
                    p->v[q] += 0.5 * dt * F[3 * k + q];
                    v2sum += p->v[q] * p->v[q];
                }
                v2n += 3;
            }
    }
    free(F);
    S->md_step += (uint64_t)nsteps;
    /* the cells of the next sweep start from this global order */
    S->E = orc_energy(S);
    return v2n ? v2sum / (double)v2n : 0.0;
}

/* ------------------------------------------------------------------------- */
/* Paper schedule: global moves                                               */
/* ------------------------------------------------------------------------- */
/* series: one row [nA-, nB+, nX+, nX-] every sample_every trials */
int orc_paper_trials(orc_sys* S, int64_t ntrials, int64_t sample_every, int32_t* series)
{
    orc_dom D;
    memset(&D, 0, sizeof D);
    D.paper = 1;
    D.ncell = 1;
    D.nreact = 3;
    D.react[0] = 0; D.react[1] = 1; D.react[2] = 2;
    D.lnZ[0] = log(S->rho0NA * S->L * S->L * S->L);
    orc_list whole;
    int64_t cnt[6];
    int64_t row = 0;
    for (int64_t t = 0; t < ntrials; ++t) {
        uint32_t w[24];
        int64_t g = S->paper_trial++;
        trial_words(S, TAG_PAPER, (uint32_t)g, (uint32_t)(g >> 32), 0u, w);
        whole.n = S->np; whole.cap = S->npcap; whole.p = S->P;
        D.list[0] = &whole;
        do_trial(S, &D, w, -1, g, 0);
        S->np = whole.n; S->npcap = whole.cap; S->P = whole.p;
        if (series && sample_every > 0 && (t + 1) % sample_every == 0) {
            orc_counts(S, cnt);
            series[4 * row + 0] = (int32_t)cnt[1]; series[4 * row + 1] = (int32_t)cnt[3];
            series[4 * row + 2] = (int32_t)cnt[4]; series[4 * row + 3] = (int32_t)cnt[5];
            ++row;
        }
    }
    return 0;
}
