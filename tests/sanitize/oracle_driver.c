/* Exercises the oracle's C entry points (cell and paper schedules, learned
   proposal, relocation trials, test aids, ungrouping, network gradient and
   Adam) for a build with AddressSanitizer and UndefinedBehaviorSanitizer.
   Exit status 0 when every call returned as expected. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_sys orc_sys;
orc_sys* orc_create(double L, int n_cells, double lB, double kappa, double rc, double eps, double rho0NA,
                    int ion_coupling, uint64_t seed, uint32_t replica);
void orc_destroy(orc_sys* S);
void orc_set_conditions(orc_sys* S, double pH, double pKa, double pKb, double pIXp, double pIXm, double pKw);
void orc_set_schedule(orc_sys* S, int trials, int fixed_grid, int pairing, int site_trials);
void orc_set_ion_trials(orc_sys* S, int n);
int orc_set_particles(orc_sys* S, int np, const uint32_t* xyz, const int32_t* kind, const int32_t* charged,
                      const int32_t* sid);
int orc_set_cores(orc_sys* S, int nc, const uint32_t* xyz, const double* radius);
int orc_sweeps(orc_sys* S, int64_t n, int32_t* series);
int orc_paper_trials(orc_sys* S, int64_t n, int64_t every, int32_t* series);
int orc_num_particles(const orc_sys* S);
int orc_get_particles(const orc_sys* S, int cap, uint32_t* xyz, int32_t* kind, int32_t* charged, int32_t* sid);
int orc_load_state(orc_sys* S, int np, const uint32_t* xyz, const int32_t* kind, const int32_t* charged,
                   const int32_t* sid, uint64_t sweep, int with_energy);
void orc_prepare_sweep(orc_sys* S);
void orc_set_domain_filter(orc_sys* S, int n, const int32_t* cells);
void orc_set_trial_limit(orc_sys* S, int64_t n);
void orc_set_check(orc_sys* S, int on);
double orc_max_dU_err(const orc_sys* S);
int orc_mlp_params(void);
int orc_set_learned(orc_sys* S, const double* par, double eps, int on);
int orc_features_of_cell_sites(const orc_sys* S, int c, int cap, int32_t* sid, double* X);
double orc_mlp_loss_grad(const double* par, const double* X, const double* y, int n, double* grad);
void orc_adam_step(double* par, const double* grad, double* m, double* v, int64_t t, double lr, double b1,
                   double b2, double eps);
void orc_ungroup(const orc_sys* S, const double frac[4], uint64_t draw, int64_t counts[6], int32_t* labels);
double orc_energy(const orc_sys* S);

static uint64_t st = 88172645463325252ull;
static uint32_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (uint32_t)st; }

int main(void)
{
    const double L = 24.0;
    enum { NP = 60 };
    uint32_t xyz[3 * NP];
    int32_t kind[NP];
    for (int i = 0; i < NP; ++i) {
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = rnd();
        kind[i] = i < 20 ? 1 : (i < 35 ? 2 : (i < 48 ? 3 : 4));
    }
    uint32_t core[3] = {1u << 31, 1u << 31, 1u << 31};
    double R = 2.0;
    orc_sys* S = orc_create(L, 4, 2.0, 0.5, 6.0, 1.0, 0.0269424, 1, 77, 1);
    orc_set_conditions(S, 6.0, 5.0, 5.0, 0.5, 0.7, 14.0);
    orc_set_particles(S, NP, xyz, kind, NULL, NULL);
    orc_set_cores(S, 1, core, &R);
    orc_set_schedule(S, 3, 0, 1, 8);
    orc_set_ion_trials(S, 1);
    orc_set_check(S, 1);
    const int P = orc_mlp_params();
    double* par = calloc((size_t)P, sizeof(double));
    for (int i = 0; i < P; ++i) par[i] = ((double)(rnd() >> 8) / 16777216.0 - 0.5) * 0.4;
    if (orc_set_learned(S, par, 0.3, 1) != 0) return 2;
    int32_t series[4 * 50];
    orc_sweeps(S, 20, series);
    if (!(orc_max_dU_err(S) < 1e-9)) return 3;
    int n = orc_num_particles(S);
    uint32_t* X = malloc(sizeof(uint32_t) * 3 * (size_t)n);
    int32_t *k = malloc(sizeof(int32_t) * (size_t)n), *c = malloc(sizeof(int32_t) * (size_t)n),
            *s = malloc(sizeof(int32_t) * (size_t)n);
    orc_get_particles(S, n, X, k, c, s);
    orc_sys* T = orc_create(L, 4, 2.0, 0.5, 6.0, 1.0, 0.0269424, 1, 77, 1);
    orc_set_conditions(T, 6.0, 5.0, 5.0, 0.5, 0.7, 14.0);
    orc_set_cores(T, 1, core, &R);
    orc_load_state(T, n, X, k, c, s, 20, 1);
    orc_set_learned(T, par, 0.3, 1);
    orc_prepare_sweep(T);
    int32_t sid[256];
    double F[256 * 32];
    for (int cc = 0; cc < 64; ++cc) orc_features_of_cell_sites(T, cc, 256, sid, F);
    int32_t pick[2] = {0, 2};
    orc_set_domain_filter(T, 2, pick);
    orc_sweeps(T, 1, NULL);
    orc_set_domain_filter(T, -1, NULL);
    orc_set_trial_limit(T, 50);
    orc_sweeps(T, 2, NULL);
    orc_set_trial_limit(T, -1);
    double frac[4] = {0.6, 0.4, 0.3, 0.5};
    int64_t cnt[6];
    int32_t* lab = malloc(sizeof(int32_t) * (size_t)orc_num_particles(T));
    orc_ungroup(T, frac, 12345, cnt, lab);
    orc_paper_trials(S, 5000, 100, series);
    /* network gradient and one Adam step */
    double Xr[8 * 32], y[8], *grad = calloc((size_t)P, sizeof(double)),
           *m = calloc((size_t)P, sizeof(double)), *v = calloc((size_t)P, sizeof(double));
    for (int i = 0; i < 8 * 32; ++i) Xr[i] = (double)(rnd() % 7);
    for (int i = 0; i < 8; ++i) y[i] = (double)(rnd() & 1);
    const double loss = orc_mlp_loss_grad(par, Xr, y, 8, grad);
    orc_adam_step(par, grad, m, v, 1, 1e-3, 0.9, 0.999, 1e-8);
    if (!isfinite(loss) || !isfinite(orc_energy(T))) return 4;
    orc_destroy(S);
    orc_destroy(T);
    free(par); free(X); free(k); free(c); free(s); free(lab); free(grad); free(m); free(v);
    printf("oracle driver ok\n");
    return 0;
}
