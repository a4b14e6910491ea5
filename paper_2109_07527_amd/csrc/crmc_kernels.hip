// CDNA4 (gfx950) kernels of the CR-MC hot path.
//
//   k_bin        per sweep: draw the grid shift, re-bin every record into the
//                shifted cells (stable: old cell order, then order in the old
//                cell), sample per-site occupancy, publish the sweep's shift and
//                pairing table.  One wavefront per new cell gathers from the old
//                cells that overlap it (at most 27, usually 8): no atomics, no scan.
//   k_phase<R>   per colour: one 256-thread workgroup per domain (one cell, or
//                two reflection-paired cells of the colour).  Stages the
//                domain's cells and their 26-cell neighbourhoods in LDS, then
//                runs the domain's trials back to back: Philox words, move and
//                participants, pair sum of the energy change over the staged
//                records (R = float or double terms, FP64 accumulation,
//                wavefront + workgroup reduction), acceptance of Sec. II C,
//                commit in LDS.  Writes the cells back at the end.
//   k_sweep_end  per sweep: series row, group histograms, sweep counter.
//   k_energy     total energy of a replica from scratch (FP64), per cell.
#include "crmc_internal.h"

#include <math.h>

namespace crmc {

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ------------------------------------------------------------------------
// integer helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pick32(uint32_t w, uint32_t m) { return __umulhi(w, m); }

__device__ __forceinline__ uint32_t pick64(uint32_t hi, uint32_t lo, uint32_t m)
{
    const uint64_t top = (uint64_t)hi * m + (uint64_t)__umulhi(lo, m);
    return (uint32_t)(top >> 32);
}

__device__ __forceinline__ double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint32_t cell_of(uint32_t y, uint32_t n) { return __umulhi(y, n); }

__device__ __forceinline__ void grid_shift(uint32_t k0, uint32_t k1, uint64_t sweep, int fixed, uint32_t o[3])
{
    if (fixed) { o[0] = o[1] = o[2] = 0u; return; }
    uint32_t w[4];
    philox4x32_10((uint32_t)sweep, 0u, 0u, TAG_SHIFT, k0, k1, w);
    o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
}

__device__ __forceinline__ int rec_kind(uint32_t meta) { return (int)(meta & 7u); }
__device__ __forceinline__ int rec_charged(uint32_t meta) { return (int)((meta >> 3) & 1u); }
__device__ __forceinline__ int rec_is_ion(uint32_t meta)
{
    const uint32_t k = meta & 7u;
    return k == KIND_XPOS || k == KIND_XNEG;
}
__device__ __forceinline__ int rec_q(uint32_t meta)
{
    const uint32_t k = meta & 7u, c = (meta >> 3) & 1u;
    if (k == KIND_ACID) return -(int)c;
    if (k == KIND_BASE) return (int)c;
    if (k == KIND_XPOS) return 1;
    if (k == KIND_XNEG) return -1;
    return 0;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = threadIdx.x & 63u;
    return lane ? (~0ull >> (64u - lane)) : 0ull;
}

// ------------------------------------------------------------------------
// k_bin: stable re-binning into the shifted grid of this sweep
// ------------------------------------------------------------------------
__global__ __launch_bounds__(BIN_THREADS) void k_bin(SweepArgs a)
{
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t gcell = blockIdx.x * (BIN_THREADS / 64) + wave;
    if (gcell >= a.ncell_total) return;
    const uint32_t r = a.cell2rep[gcell];
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, cap = R.cap;
    const uint32_t k = gcell - R.cell_begin;
    const uint64_t s = *a.sweep;
    const int cur = (int)(s & 1u), nxt = cur ^ 1;
    const uint4* __restrict__ src = R.rec[cur];
    const uint32_t* __restrict__ scnt = R.cnt[cur];
    uint4* __restrict__ dst = R.rec[nxt];
    const uint32_t* __restrict__ bnd = R.bnd;
    const uint32_t hw = *R.hiwater;

    uint32_t on[3], oo[3];
    grid_shift(R.key0, R.key1, s, a.fixed_grid, on);
    if (s == 0) { oo[0] = oo[1] = oo[2] = 0u; }
    else grid_shift(R.key0, R.key1, s - 1, a.fixed_grid, oo);

    if (k == 0 && lane < 12) {
        // the sweep's table: shift, and the pairing centre of every colour
        const uint32_t M = R.h * R.h * R.h;
        uint32_t v = 0;
        if (lane < 4) v = lane < 3 ? on[lane] : 0u;
        else {
            uint32_t w[4];
            philox4x32_10((uint32_t)s, lane - 4u, 0u, TAG_PAIR, R.key0, R.key1, w);
            const uint32_t rr = pick32(w[0], M);
            v = (uint32_t)(((uint64_t)M - 1u + 2ull * M - 2ull * rr) % M);
        }
        if (lane < 4) R.tab->o[lane] = v; else R.tab->pairc[lane - 4] = v;
    }

    const uint32_t kc[3] = {k % n, (k / n) % n, k / (n * n)};
    uint32_t cand[3][3];
    int ncand[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t lo_abs = on[d] + bnd[kc[d]];
        const uint32_t hi_abs = on[d] + bnd[kc[d] + 1] - 1u;
        const uint32_t j0 = cell_of(lo_abs - oo[d], n), j1 = cell_of(hi_abs - oo[d], n);
        const int m = (int)((j1 + n - j0) % n) + 1;
        uint32_t v0 = j0, v1 = (j0 + 1u) % n, v2 = (j0 + 2u) % n;
        // ascending order (a wrap-around puts small indices last)
        if (m == 2 && v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
        if (m == 3) {
            if (v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
            if (v2 < v1) { uint32_t t = v1; v1 = v2; v2 = t; }
            if (v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
        }
        cand[d][0] = v0; cand[d][1] = v1; cand[d][2] = v2;
        ncand[d] = m;
    }

    const uint64_t lt = lanemask_lt();
    uint32_t base = 0;
    for (int iz = 0; iz < ncand[2]; ++iz)
        for (int iy = 0; iy < ncand[1]; ++iy)
            for (int ix = 0; ix < ncand[0]; ++ix) {
                const uint32_t oc = cand[0][ix] + n * (cand[1][iy] + n * cand[2][iz]);
                const uint32_t cc = scnt[oc];
                for (uint32_t b = 0; b < cc; b += 64u) {
                    const uint32_t i = b + lane;
                    bool match = false;
                    uint4 rec = make_uint4(0, 0, 0, 0);
                    if (i < cc) {
                        rec = src[(size_t)oc * cap + i];
                        match = cell_of(rec.x - on[0], n) == kc[0] && cell_of(rec.y - on[1], n) == kc[1] &&
                                cell_of(rec.z - on[2], n) == kc[2];
                    }
                    const uint64_t mask = __ballot(match);
                    if (match) {
                        const uint32_t pos = base + (uint32_t)__popcll(mask & lt);
                        if (pos < cap) dst[(size_t)k * cap + pos] = rec;
                        const uint32_t sid = rec.w >> 8;
                        // each site lands in exactly one new cell: non-returning adds
                        if (sid != NO_SITE && rec_charged(rec.w)) {
                            atomicAdd((unsigned long long*)&R.occupancy[sid], 1ull);
                            atomicAdd(&R.group_count[(s & 1u) * R.ngroups + (uint32_t)R.site_group[sid]], 1);
                        }
                    }
                    base += (uint32_t)__popcll(mask);
                }
            }
    if (lane == 0) {
        R.cnt[nxt][k] = base < cap ? base : cap;
        R.cnt0[k] = base < cap ? base : cap;
        if (base > cap) atomicOr(a.err, ERR_BIN_CAPACITY);
        if (base > hw) atomicMax(R.hiwater, base); // rarely taken once the mark has settled
    }
}

// ------------------------------------------------------------------------
// precision policy of the pair terms
// ------------------------------------------------------------------------
template <typename Real> struct Math;
template <> struct Math<float> {
    __device__ static __forceinline__ float rsqrt(float x) { return rsqrtf(x); }
    __device__ static __forceinline__ float ex(float x) { return __expf(x); }
    __device__ static __forceinline__ float rcp(float x) { return __frcp_rn(x); }
    __device__ static __forceinline__ float sqrt_(float x) { return sqrtf(x); }
};
template <> struct Math<double> {
    __device__ static __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
    __device__ static __forceinline__ double ex(double x) { return exp(x); }
    __device__ static __forceinline__ double rcp(double x) { return 1.0 / x; }
    __device__ static __forceinline__ double sqrt_(double x) { return sqrt(x); }
};

// a particle whose state the trial changes
struct Chg {
    uint32_t x, y, z;
    int dq;      // charge change seen by every other particle
    int dw;      // +1 inserted free ion, -1 deleted free ion, 0 otherwise
    int member;  // domain cell it lives in
    int own;     // index in that cell's list, -1 if inserted
    int q_old, q_new, ion, pres_old, pres_new;
};

struct PairParams {
    float scale_f;
    double scale_d;
    uint64_t R2;
    double rc2_lo, rc2_hi; // rc^2 (1 -+ 1e-5): outside this band the float distance decides
    double lB, kappa, eps;
    int ion_coupling;
};

template <typename Real>
__device__ __forceinline__ Real scale_of(const PairParams& P)
{
    return sizeof(Real) == 4 ? (Real)P.scale_f : (Real)P.scale_d;
}

template <typename Real>
__device__ __forceinline__ double pair_term(const uint4& rec, const Chg& c, const PairParams& P, int& ov)
{
    // distance first: most records of a 27-cell neighbourhood lie beyond rc
    const int32_t dx = (int32_t)(rec.x - c.x), dy = (int32_t)(rec.y - c.y), dz = (int32_t)(rec.z - c.z);
    const Real sc = scale_of<Real>(P);
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r2 = fx * fx + fy * fy + fz * fz;
    if (r2 > (Real)P.rc2_hi) return 0.0;
    const int ionj = rec_is_ion(rec.w);
    if (!P.ion_coupling && ionj) return 0.0;
    const int qj = rec_q(rec.w);
    const bool coul = c.dq != 0 && qj != 0;
    const bool ev = c.dw != 0;
    if (!coul && !ev) return 0.0;
    double e = 0.0;
    if (coul) {
        // inside/outside the cutoff as decided on the exact integer squared
        // distance; the float distance settles it outside a +-1e-5 band
        bool in = r2 < (Real)P.rc2_lo;
        if (!in) {
            const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
            const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
            in = r2i < P.R2;
        }
        if (in) {
            const Real rinv = Math<Real>::rsqrt(r2);
            const Real r = r2 * rinv;
            const Real phi = Math<Real>::ex(-(Real)P.kappa * r) * rinv;
            e += P.lB * (double)(c.dq * qj) * (double)phi;
        }
    }
    if (ev && r2 < (Real)1.2599210498948731647672106) {
        if (r2 < (Real)0.25) {
            if (c.dw > 0) ov = 1;
        } else {
            const Real ir2 = Math<Real>::rcp(r2);
            const Real ir6 = ir2 * ir2 * ir2;
            const Real w = (Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps;
            e += (double)c.dw * (double)w;
        }
    }
    return e;
}

template <typename Real>
__device__ __forceinline__ double wca_core(const Chg& c, const uint4& cx, double delta, const PairParams& P, int& ov)
{
    const int32_t dx = (int32_t)(cx.x - c.x), dy = (int32_t)(cx.y - c.y), dz = (int32_t)(cx.z - c.z);
    const Real sc = scale_of<Real>(P);
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r = Math<Real>::sqrt_(fx * fx + fy * fy + fz * fz);
    const Real sh = r - (Real)delta;
    if (!(sh < (Real)1.122462048309373)) return 0.0;
    if (sh < (Real)0.5) {
        if (c.dw > 0) ov = 1;
        return 0.0;
    }
    const Real ir2 = Math<Real>::rcp(sh * sh);
    const Real ir6 = ir2 * ir2 * ir2;
    return (double)c.dw * (double)((Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps);
}

// the pair formed or broken between the two changed particles
template <typename Real>
__device__ __forceinline__ double changed_pair(const Chg& A, const Chg& B, const PairParams& P, bool ev_on, int& ov)
{
    if (!P.ion_coupling && (A.ion || B.ion)) return 0.0;
    const int32_t dx = (int32_t)(B.x - A.x), dy = (int32_t)(B.y - A.y), dz = (int32_t)(B.z - A.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const Real sc = scale_of<Real>(P);
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r2 = fx * fx + fy * fy + fz * fz;
    double e = 0.0;
    const int dqq = A.q_new * B.q_new - A.q_old * B.q_old;
    if (dqq != 0 && r2i < P.R2) {
        const Real rinv = Math<Real>::rsqrt(r2);
        e += P.lB * (double)dqq * (double)(Math<Real>::ex(-(Real)P.kappa * r2 * rinv) * rinv);
    }
    const int any_ion = A.ion || B.ion;
    const int pn = ev_on && any_ion && A.pres_new && B.pres_new;
    const int po = ev_on && any_ion && A.pres_old && B.pres_old;
    if ((pn || po) && r2 < (Real)1.2599210498948731647672106) {
        if (r2 < (Real)0.25) {
            if (pn) ov = 1;
        } else {
            const Real ir2 = Math<Real>::rcp(r2);
            const Real ir6 = ir2 * ir2 * ir2;
            e += (double)(pn - po) * (double)((Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps);
        }
    }
    return e;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------------
// k_phase: one colour of one sweep
// ------------------------------------------------------------------------
constexpr int MAX_LDS_CORES = 64; // nanoparticle cores held on chip (more are read from memory)

struct PhaseShared {
    int32_t pre[53];       // prefix of the 52 neighbour segments (member 0, then 1)
    uint32_t seg_cell[52]; // neighbour cell of each segment
    double red[2][8];      // per wavefront partial sums (up to eight wavefronts), two trials deep
    int32_t ovf[2][8];
    uint32_t att[6], acc[6];
    int32_t dtot[4];
    uint4 core[MAX_LDS_CORES];
    double core_delta[MAX_LDS_CORES];
};

// position g of the concatenated neighbour segments -> segment
__device__ __forceinline__ int segment_of(const PhaseShared& S, int g)
{
    int lo = 0, hi = 52; // pre[lo] <= g < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (S.pre[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint4 neighbour_global(const PhaseShared& S, const uint4* recb, uint32_t cap, int g)
{
    const int q = segment_of(S, g);
    return recb[(size_t)S.seg_cell[q] * cap + (uint32_t)(g - S.pre[q])];
}

// LDS pool layout of a domain (offsets in records of smem):
//   [0, room0) member 0's list | [room0, room0+room1) member 1's list |
//   ln k table (doubles) | neighbour records (when they fit)
struct Pool {
    int room0, room1, ln_off, nb_off;
    __device__ __forceinline__ int base(int member) const { return member ? room0 : 0; }
};

extern __shared__ uint4 smem[];

// domain-order index of the k-th record of the domain matching the predicate
// (member 0's list, then member 1's); each wavefront computes it alone
template <typename Pred>
__device__ __forceinline__ int domain_kth(const Pool& pl, int n0, int n1, Pred pred, int k)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt();
    const int total = n0 + n1;
    for (int b = 0; b < total; b += 64) {
        const int g = b + lane;
        bool p = false;
        if (g < total) p = pred(smem[g < n0 ? g : pl.room0 + (g - n0)].w);
        const uint64_t mask = __ballot(p);
        const int cnt = __popcll(mask);
        if (k < cnt) {
            const bool mine = p && __popcll(mask & lt) == k;
            const uint64_t hit = __ballot(mine);
            return b + (__ffsll((long long)hit) - 1);
        }
        k -= cnt;
    }
    return -1;
}

template <typename Real, int NT>
__global__ __launch_bounds__(NT) void k_phase(SweepArgs a)
{
    __shared__ PhaseShared S;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t t_start = a.trace ? wall_clock64() : 0;
    const uint32_t gd = blockIdx.x;
    // the replica is uniform over the workgroup: keep its constants in scalar registers
    const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.dom2rep[gd]);
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, h = R.h, cap = R.cap;
    const uint64_t s = *a.sweep;
    const int buf = (int)((s + 1u) & 1u);
    uint4* __restrict__ recb = R.rec[buf];
    uint32_t* __restrict__ cntb = R.cnt[buf];
    const uint32_t key0 = R.key0, key1 = R.key1;
    const uint32_t ncores = R.ncores;
    const uint4* __restrict__ core_g = R.core_x;
    const double* __restrict__ cdel_g = R.core_delta;
    const int colour = a.colour;
    const uint32_t px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;

    // ---- the domain of this workgroup -------------------------------------
    const uint32_t M = h * h * h;
    const uint32_t d = gd - R.dom_begin;
    uint32_t ma, mb;
    if (a.pairing) {
        const uint32_t c = R.tab->pairc[colour];
        const uint32_t half = c >> 1;
        if (d <= half) { ma = d; mb = c - d; }
        else { ma = c + 1u + (d - half - 1u); mb = M + c - ma; }
    } else {
        ma = mb = d;
    }
    const int ncell = (ma == mb) ? 1 : 2;
    uint32_t cc0[3], cc1[3];
    cc0[0] = 2u * (ma % h) + px; cc0[1] = 2u * ((ma / h) % h) + py; cc0[2] = 2u * (ma / (h * h)) + pz;
    cc1[0] = 2u * (mb % h) + px; cc1[1] = 2u * ((mb / h) % h) + py; cc1[2] = 2u * (mb / (h * h)) + pz;
    const uint32_t cell0 = cc0[0] + n * (cc0[1] + n * cc0[2]);
    const uint32_t cell1 = cc1[0] + n * (cc1[1] + n * cc1[2]);

    // the LDS pool: each member's list with room for the growth its trials can
    // cause (two ions per trial, the site count bounded by the record count),
    // the ln k table for every count the domain can reach, then the neighbours
    // (the binned counts: cells of this colour are changed by this phase only)
    int n0 = (int)R.cnt0[cell0];
    int n1 = ncell == 2 ? (int)R.cnt0[cell1] : 0;
    const int ntr_max = a.trials * ncell + ((n0 + n1) * a.site_trials + 15) / 16;
    Pool pl;
    pl.room0 = min((int)cap, n0 + 2 * ntr_max);
    pl.room1 = ncell == 2 ? min((int)cap, n1 + 2 * ntr_max) : 0;
    const int nln = pl.room0 + pl.room1 + 2; // ln k for k < nln
    pl.ln_off = pl.room0 + pl.room1;
    pl.nb_off = pl.ln_off + (nln + 1) / 2;
    double* lnt = reinterpret_cast<double*>(smem + pl.ln_off);

    // ---- neighbour segments: counts, then a wavefront prefix scan -----------
    if (wave == 0) {
        int cnt = 0;
        uint32_t nc = 0;
        if (lane < 52) {
            const int j = lane / 26, q = lane % 26;
            const int o = q < 13 ? q : q + 1;
            const uint32_t* cc = j ? cc1 : cc0;
            if (j < ncell) {
                const uint32_t x = (cc[0] + n + (uint32_t)(o % 3) - 1u) % n;
                const uint32_t y = (cc[1] + n + (uint32_t)((o / 3) % 3) - 1u) % n;
                const uint32_t z = (cc[2] + n + (uint32_t)(o / 9) - 1u) % n;
                nc = x + n * (y + n * z);
                cnt = (int)cntb[nc];
            }
            S.seg_cell[lane] = nc;
        }
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (lane < 52) S.pre[lane + 1] = incl;
        if (lane == 0) S.pre[0] = 0;
    }
    if (tid < 6) { S.att[tid] = 0; S.acc[tid] = 0; }
    if (tid < 4) S.dtot[tid] = 0;
    __syncthreads();
    const int nb_total = S.pre[52];
    // A split launch takes one class of domains: light ones, whose lists, ln
    // table and neighbours fit the small pool, go to a one-wavefront launch,
    // the others to a wide one.  The decision uses the binned counts of the
    // domain's cells and the counts of its neighbours (inactive cells), none of
    // which any workgroup of this phase modifies, so both launches agree.
    const int need = pl.nb_off + nb_total;
    if ((a.cls == 1 && need > a.split) || (a.cls == 2 && need <= a.split)) return;
    for (int i = tid; i < n0; i += NT) smem[i] = recb[(size_t)cell0 * cap + i];
    for (int i = tid; i < n1; i += NT) smem[pl.room0 + i] = recb[(size_t)cell1 * cap + i];
    for (int i = tid; i < nln; i += NT) lnt[i] = a.lntab[i];
    for (int i = tid; i < (int)min(ncores, (uint32_t)MAX_LDS_CORES); i += NT) {
        S.core[i] = core_g[i];
        S.core_delta[i] = cdel_g[i];
    }
    const bool staged = pl.nb_off + nb_total <= a.budget;
    if (staged) {
        for (int g = tid; g < nb_total; g += NT) {
            const int q = segment_of(S, g);
            smem[pl.nb_off + g] = recb[(size_t)S.seg_cell[q] * cap + (uint32_t)(g - S.pre[q])];
        }
    } else if (tid == 0) {
        atomicOr(a.err, INFO_UNSTAGED);
    }
    const int nbc0 = S.pre[26];
    const int nbb1 = S.pre[26], nbc1 = S.pre[52] - S.pre[26];
    __syncthreads();

    // ---- counts of the domain, one pass -------------------------------------
    int m0a = 0, mca = 0, m0b = 0, mcb = 0, npos = 0, nneg = 0;
    {
        const int total = n0 + n1;
        for (int b = 0; b < total; b += 64) {
            const int g = b + lane;
            uint32_t m = 0;
            if (g < total) m = smem[g < n0 ? g : pl.room0 + (g - n0)].w;
            const int kd = g < total ? rec_kind(m) : 0, ch = rec_charged(m);
            m0a += __popcll(__ballot(kd == (int)KIND_ACID && !ch));
            mca += __popcll(__ballot(kd == (int)KIND_ACID && ch));
            m0b += __popcll(__ballot(kd == (int)KIND_BASE && !ch));
            mcb += __popcll(__ballot(kd == (int)KIND_BASE && ch));
            npos += __popcll(__ballot(kd == (int)KIND_XPOS));
            nneg += __popcll(__ballot(kd == (int)KIND_XNEG));
        }
    }
    // trials of this domain: the state-independent schedule
    const int ntr = a.trials * ncell + ((m0a + mca + m0b + mcb) * a.site_trials + 15) / 16;
    int react0 = 2, react1 = 2;
    int nreact = 1;
    {
        const bool ha = m0a + mca > 0, hb = m0b + mcb > 0;
        if (ha && hb) { react0 = 0; react1 = 1; nreact = 3; }
        else if (ha) { react0 = 0; nreact = 2; }
        else if (hb) { react0 = 1; nreact = 2; }
    }

    // insertion regions and volume terms of the members (tables built on the host)
    const uint32_t o0 = R.tab->o[0], o1 = R.tab->o[1], o2 = R.tab->o[2];
    const uint32_t* bnd = R.bnd;
    const double lnk = ncell == 2 ? a.ln2 : 0.0;
    uint32_t ib0[3], iw0[3], ib1[3], iw1[3];
    {
        const uint32_t oo[3] = {o0, o1, o2};
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            const uint32_t l0 = bnd[cc0[dd]], h0 = bnd[cc0[dd] + 1];
            const uint32_t l1 = bnd[cc1[dd]], h1 = bnd[cc1[dd] + 1];
            ib0[dd] = oo[dd] + l0; iw0[dd] = h0 - l0;
            ib1[dd] = oo[dd] + l1; iw1[dd] = h1 - l1;
        }
    }
    const double lnZm0 = (R.lnZ0 + lnk) + ((R.lnW[cc0[0]] + R.lnW[cc0[1]]) + R.lnW[cc0[2]]);
    const double lnZm1 = (R.lnZ0 + lnk) + ((R.lnW[cc1[0]] + R.lnW[cc1[1]]) + R.lnW[cc1[2]]);

    PairParams P;
    P.scale_f = (float)R.scale;
    P.scale_d = R.scale;
    P.R2 = R.R2;
    P.rc2_lo = (double)R.R2 * R.scale * R.scale * (1.0 - 1e-5);
    P.rc2_hi = (double)R.R2 * R.scale * R.scale * (1.0 + 1e-5);
    P.lB = a.lB;
    P.kappa = R.kappa;
    P.eps = a.eps;
    P.ion_coupling = a.ion_coupling;
    const bool ev_on = a.eps > 0.0 && a.ion_coupling;
    const double lnKA = R.lnKA, lnKB = R.lnKB, lnKion = R.lnKion;

    double dE = 0.0;
    for (int t = 0; t < ntr; ++t) {
        // 20 Philox words: lane b of every wavefront computes block b
        uint32_t wl[4];
        philox4x32_10((uint32_t)s, cell0, (uint32_t)t * 8u + (uint32_t)(lane < 5 ? lane : 0), TAG_TRIAL,
                      key0, key1, wl);
        uint32_t W[20];
#pragma unroll
        for (int i = 0; i < 20; ++i) W[i] = (uint32_t)__builtin_amdgcn_readlane((int)wl[i & 3], i >> 2);

        const uint32_t kk = pick32(W[0], (uint32_t)(2 * nreact));
        const int rsel = (int)(kk >> 1);
        const int reaction = rsel == 0 ? react0 : (rsel == 1 ? react1 : 2);
        const int move = 2 * reaction + (int)(kk & 1u);
        const double u = unit53(W[16], W[17]);

        // participants: A is the site (moves 0-3) or the cation (4, 5); B is the ion
        int a_idx = -1, b_idx = -1; // domain-order indices of existing participants
        bool auto_reject = false;
        double lnp_counts = 0.0;
        switch (move) {
        case 0:
            if (m0a == 0) { auto_reject = true; break; }
            a_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_ACID && !rec_charged(m); },
                               (int)pick32(W[1], (uint32_t)m0a));
            lnp_counts = lnt[m0a] - lnt[mca + 1] - lnt[npos + 1] + lnKA;
            break;
        case 1:
            if (mca == 0 || npos == 0) { auto_reject = true; break; }
            a_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_ACID && rec_charged(m); },
                               (int)pick32(W[1], (uint32_t)mca));
            b_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XPOS; },
                               (int)pick32(W[2], (uint32_t)npos));
            lnp_counts = lnt[mca] + lnt[npos] - lnt[m0a + 1] - lnKA;
            break;
        case 2:
            if (m0b == 0) { auto_reject = true; break; }
            a_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_BASE && !rec_charged(m); },
                               (int)pick32(W[1], (uint32_t)m0b));
            lnp_counts = lnt[m0b] - lnt[mcb + 1] - lnt[nneg + 1] + lnKB;
            break;
        case 3:
            if (mcb == 0 || nneg == 0) { auto_reject = true; break; }
            a_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_BASE && rec_charged(m); },
                               (int)pick32(W[1], (uint32_t)mcb));
            b_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XNEG; },
                               (int)pick32(W[3], (uint32_t)nneg));
            lnp_counts = lnt[mcb] + lnt[nneg] - lnt[m0b + 1] - lnKB;
            break;
        case 4:
            lnp_counts = -lnt[npos + 1] - lnt[nneg + 1] + lnKion;
            break;
        default:
            if (npos == 0 || nneg == 0) { auto_reject = true; break; }
            a_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XPOS; },
                               (int)pick32(W[2], (uint32_t)npos));
            b_idx = domain_kth(pl, n0, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XNEG; },
                               (int)pick32(W[3], (uint32_t)nneg));
            lnp_counts = lnt[npos] + lnt[nneg] - lnKion;
            break;
        }
        if (tid == 0) S.att[move] += 1u;
        if (auto_reject) {
            if (tid == 0 && a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = cell0; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = 2;
                    L.dU = __longlong_as_double(0x7FF8000000000000ll); L.lnp = L.dU; L.u = u;
                }
            }
            continue;
        }

        // ---- the two changed particles -------------------------------------
        Chg A, B;
        double lnvol = 0.0;
        if (move <= 3) {
            // A: the site flips
            A.member = a_idx < n0 ? 0 : 1;
            A.own = a_idx < n0 ? a_idx : a_idx - n0;
            const uint4 rc = smem[pl.base(A.member) + A.own];
            A.x = rc.x; A.y = rc.y; A.z = rc.z;
            const int chg = rec_charged(rc.w);
            const int sgn = rec_kind(rc.w) == (int)KIND_ACID ? -1 : 1;
            A.q_old = sgn * chg; A.q_new = sgn * (1 - chg);
            A.dq = A.q_new - A.q_old; A.dw = 0; A.ion = 0; A.pres_old = 1; A.pres_new = 1;
        }
        const bool insertion = move == 0 || move == 2 || move == 4;
        // B (and A for salt moves): ions in or out
        {
            const int qB = (move <= 1) ? 1 : -1; // cation for acid moves, anion otherwise
            B.ion = 1;
            B.q_old = insertion ? 0 : qB;
            B.q_new = insertion ? qB : 0;
            B.pres_old = insertion ? 0 : 1;
            B.pres_new = insertion ? 1 : 0;
            B.dq = a.ion_coupling ? B.q_new - B.q_old : 0;
            B.dw = ev_on ? (insertion ? 1 : -1) : 0;
            if (insertion) {
                const uint32_t wc = qB > 0 ? W[18] : W[19];
                const int wo = qB > 0 ? 4 : 10;
                const int j = ncell == 1 ? 0 : (int)pick32(wc, (uint32_t)ncell);
                B.member = j;
                B.own = -1;
                B.x = (j ? ib1[0] : ib0[0]) + pick64(W[wo + 0], W[wo + 1], j ? iw1[0] : iw0[0]);
                B.y = (j ? ib1[1] : ib0[1]) + pick64(W[wo + 2], W[wo + 3], j ? iw1[1] : iw0[1]);
                B.z = (j ? ib1[2] : ib0[2]) + pick64(W[wo + 4], W[wo + 5], j ? iw1[2] : iw0[2]);
                lnvol += j ? lnZm1 : lnZm0;
            } else {
                B.member = b_idx < n0 ? 0 : 1;
                B.own = b_idx < n0 ? b_idx : b_idx - n0;
                const uint4 rc = smem[pl.base(B.member) + B.own];
                B.x = rc.x; B.y = rc.y; B.z = rc.z;
                lnvol -= B.member ? lnZm1 : lnZm0;
            }
        }
        if (move >= 4) {
            A.ion = 1;
            A.q_old = insertion ? 0 : 1;
            A.q_new = insertion ? 1 : 0;
            A.pres_old = insertion ? 0 : 1;
            A.pres_new = insertion ? 1 : 0;
            A.dq = a.ion_coupling ? A.q_new - A.q_old : 0;
            A.dw = ev_on ? (insertion ? 1 : -1) : 0;
            if (insertion) {
                const int j = ncell == 1 ? 0 : (int)pick32(W[18], (uint32_t)ncell);
                A.member = j;
                A.own = -1;
                A.x = (j ? ib1[0] : ib0[0]) + pick64(W[4], W[5], j ? iw1[0] : iw0[0]);
                A.y = (j ? ib1[1] : ib0[1]) + pick64(W[6], W[7], j ? iw1[1] : iw0[1]);
                A.z = (j ? ib1[2] : ib0[2]) + pick64(W[8], W[9], j ? iw1[2] : iw0[2]);
                lnvol += j ? lnZm1 : lnZm0;
            } else {
                A.member = a_idx < n0 ? 0 : 1;
                A.own = a_idx < n0 ? a_idx : a_idx - n0;
                const uint4 rc = smem[pl.base(A.member) + A.own];
                A.x = rc.x; A.y = rc.y; A.z = rc.z;
                lnvol -= A.member ? lnZm1 : lnZm0;
            }
        }
        // per-member growth check against the cell capacity
        const int gA = A.pres_new - A.pres_old, gB = B.pres_new - B.pres_old;
        const int grow0 = (A.member == 0 ? gA : 0) + (B.member == 0 ? gB : 0);
        const int grow1 = (A.member == 1 ? gA : 0) + (B.member == 1 ? gB : 0);
        const bool cap_fail = n0 + grow0 > (int)cap || n1 + grow1 > (int)cap;

        // ---- energy change: every wavefront sums a share of the records ------
        double acc = 0.0;
        int ov = 0;
        for (int j = 0; j < ncell; ++j) {
            const bool inA = A.member == j, inB = B.member == j;
            if (!inA && !inB) continue;
            const int obase = pl.base(j);
            const int no = j ? n1 : n0;
            const int skipA = inA ? A.own : -1, skipB = inB ? B.own : -1;
            const int nbb = j ? nbb1 : 0, nbc = j ? nbc1 : nbc0;
            const int total = no + nbc;
            for (int g = tid; g < total; g += NT) {
                uint4 rc;
                if (g < no) {
                    if (g == skipA || g == skipB) continue;
                    rc = smem[obase + g];
                } else {
                    const int q = nbb + (g - no);
                    rc = staged ? smem[pl.nb_off + q] : neighbour_global(S, recb, cap, q);
                }
                if (inA) acc += pair_term<Real>(rc, A, P, ov);
                if (inB) acc += pair_term<Real>(rc, B, P, ov);
            }
        }
        if (ev_on && ncores) {
            for (int k = tid; k < (int)ncores; k += NT) {
                const bool lds = k < MAX_LDS_CORES;
                const uint4 cx = lds ? S.core[k] : core_g[k];
                const double dl = lds ? S.core_delta[k] : cdel_g[k];
                if (A.dw != 0) acc += wca_core<Real>(A, cx, dl, P, ov);
                if (B.dw != 0) acc += wca_core<Real>(B, cx, dl, P, ov);
            }
        }
        if (tid == 0) acc += changed_pair<Real>(A, B, P, ev_on, ov);
        const double wsum = wave_sum(acc);
        const int wov = __ballot(ov) != 0ull;
        const int par = t & 1;
        if (lane == 0) { S.red[par][wave] = wsum; S.ovf[par][wave] = wov; }
        __syncthreads();
        double dU = S.red[par][0];
        int any_ov = S.ovf[par][0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            dU += S.red[par][w];
            any_ov |= S.ovf[par][w];
        }
        if (any_ov) dU = __longlong_as_double(0x7FF0000000000000ll);
        const double lnp = lnp_counts + lnvol - dU;
        const bool accept = !cap_fail && u < exp(lnp < 0.0 ? lnp : 0.0);
        if (tid == 0) {
            if (cap_fail) atomicOr(a.err, ERR_INSERT_CAPACITY);
            if (a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = cell0; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = accept ? 1 : 0;
                    L.dU = dU; L.lnp = lnp; L.u = u;
                }
            }
        }
        if (!accept) continue;

        // ---- commit: flip; deletions (higher index first within one cell);
        //      insertions appended, cation before anion -----------------------
        if (tid == 0) {
            S.acc[move] += 1u;
            dE += dU;
            if (move <= 3) {
                uint4& rc = smem[pl.base(A.member) + A.own];
                rc.w ^= 8u;
                S.dtot[move <= 1 ? 0 : 1] += rec_charged(rc.w) ? 1 : -1;
            }
            int l0 = n0, l1 = n1;
            if (!insertion) {
                // deleted: B always; A too for the salt move
                int dm0 = B.member, di0 = B.own, dm1 = -1, di1 = -1;
                if (move == 5) {
                    // the cation (A) first unless the anion sits higher in the same cell
                    dm0 = A.member; di0 = A.own; dm1 = B.member; di1 = B.own;
                    if (dm0 == dm1 && di1 > di0) {
                        int t0 = di0; di0 = di1; di1 = t0;
                    }
                }
                {
                    int& cnt = dm0 ? l1 : l0;
                    const int bs = pl.base(dm0);
                    smem[bs + di0] = smem[bs + cnt - 1];
                    --cnt;
                }
                if (dm1 >= 0) {
                    int& cnt = dm1 ? l1 : l0;
                    const int bs = pl.base(dm1);
                    smem[bs + di1] = smem[bs + cnt - 1];
                    --cnt;
                }
            } else {
                if (move == 4) {
                    int& cnt = A.member ? l1 : l0;
                    smem[pl.base(A.member) + cnt] = make_uint4(A.x, A.y, A.z, make_meta(KIND_XPOS, 1u, NO_SITE));
                    ++cnt;
                }
                int& cnt = B.member ? l1 : l0;
                smem[pl.base(B.member) + cnt] =
                    make_uint4(B.x, B.y, B.z, make_meta(B.q_new > 0 ? KIND_XPOS : KIND_XNEG, 1u, NO_SITE));
                ++cnt;
            }
            if (move == 0 || move == 4) S.dtot[2] += 1;
            if (move == 2 || move == 4) S.dtot[3] += 1;
            if (move == 1 || move == 5) S.dtot[2] -= 1;
            if (move == 3 || move == 5) S.dtot[3] -= 1;
        }
        n0 += grow0;
        n1 += grow1;
        switch (move) {
        case 0: m0a--; mca++; npos++; break;
        case 1: m0a++; mca--; npos--; break;
        case 2: m0b--; mcb++; nneg++; break;
        case 3: m0b++; mcb--; nneg--; break;
        case 4: npos++; nneg++; break;
        default: npos--; nneg--; break;
        }
        __syncthreads();
    }

    // ---- write the domain's cells back --------------------------------------
    __syncthreads();
    for (int i = tid; i < n0; i += NT) recb[(size_t)cell0 * cap + i] = smem[i];
    for (int i = tid; i < n1; i += NT) recb[(size_t)cell1 * cap + i] = smem[pl.room0 + i];
    if (tid == 0 && a.trace) {
        const unsigned long long ti = atomicAdd(a.trace_n, 1ull);
        if (ti < a.trace_cap) {
            PhaseTrace& T = a.trace[ti];
            T.t0 = t_start;
            T.t1 = wall_clock64();
            T.sweep = (uint32_t)s; T.domain = gd; T.colour = colour; T.ntr = ntr;
            T.nb = nb_total; T.own = n0 + n1; T.staged = staged;
            T.hw = (int32_t)__smid();
        }
    }
    if (tid == 0) {
        cntb[cell0] = (uint32_t)n0;
        if (ncell == 2) cntb[cell1] = (uint32_t)n1;
        if (dE != 0.0) R.e_acc[cell0] += dE;
        for (int i = 0; i < 6; ++i) {
            if (S.att[i]) atomicAdd((unsigned long long*)&R.moves[i], (unsigned long long)S.att[i]);
            if (S.acc[i]) atomicAdd((unsigned long long*)&R.moves[6 + i], (unsigned long long)S.acc[i]);
        }
        for (int i = 0; i < 4; ++i)
            if (S.dtot[i]) atomicAdd((unsigned long long*)&R.totals[i], (unsigned long long)(long long)S.dtot[i]);
    }
}


// ------------------------------------------------------------------------
// k_sweep_end: series row, group histograms, advance the sweep counter
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sweep_end(SweepArgs a)
{
    const uint64_t s = *a.sweep;
    for (uint32_t r = 0; r < a.nrep; ++r) {
        const Replica& R = a.reps[r];
        if (threadIdx.x < 4 && R.series_cap > 0) {
            const int64_t row = (int64_t)(s % (uint64_t)R.series_cap);
            R.series[row * 4 + threadIdx.x] = (int32_t)R.totals[threadIdx.x];
        }
        // ionized sites per group at the start of this sweep (counted by the
        // re-binning); the slot is cleared for the sweep after next
        int32_t* gc = R.group_count + (s & 1u) * R.ngroups;
        for (uint32_t g = threadIdx.x; g < R.ngroups; g += blockDim.x) {
            R.group_hist[R.group_hist_off[g] + gc[g]] += 1;
            gc[g] = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *a.sweep = s + 1u;
}

// ------------------------------------------------------------------------
// k_energy: total energy of one replica from scratch, FP64, one wave per cell
// ------------------------------------------------------------------------
__device__ double pair_energy_full(const uint4& a, const uint4& b, double scale, uint64_t R2, double lB,
                                   double kappa, double eps, int ion_coupling)
{
    const int ia = rec_is_ion(a.w), ib = rec_is_ion(b.w);
    if (!ion_coupling && (ia || ib)) return 0.0;
    const int32_t dx = (int32_t)(b.x - a.x), dy = (int32_t)(b.y - a.y), dz = (int32_t)(b.z - a.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const double r2 = (double)r2i * scale * scale;
    double e = 0.0;
    if (eps > 0.0 && (ia || ib) && r2 < 1.2599210498948731647672106) {
        if (r2 < 0.25) return __longlong_as_double(0x7FF0000000000000ll);
        const double ir2 = 1.0 / r2, ir6 = ir2 * ir2 * ir2;
        e += 4.0 * eps * (ir6 * ir6 - ir6) + eps;
    }
    const int qa = rec_q(a.w), qb = rec_q(b.w);
    if (r2i < R2 && qa != 0 && qb != 0) {
        const double r = sqrt(r2);
        e += lB * (double)(qa * qb) * exp(-kappa * r) / r;
    }
    return e;
}

__global__ __launch_bounds__(64) void k_energy(const Replica* rep, int buf, double lB, double eps, int ion_coupling,
                                               double* out)
{
    const Replica& R = *rep;
    const uint32_t n = R.n, cap = R.cap;
    const uint32_t c = blockIdx.x;
    const uint32_t cx = c % n, cy = (c / n) % n, cz = c / (n * n);
    const uint4* recb = R.rec[buf];
    const uint32_t* cntb = R.cnt[buf];
    const uint32_t nc = cntb[c];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < nc; i += 64) {
        const uint4 a = recb[(size_t)c * cap + i];
        for (int o = 0; o < 27; ++o) {
            const uint32_t x = (cx + n + (uint32_t)(o % 3) - 1u) % n, y = (cy + n + (uint32_t)((o / 3) % 3) - 1u) % n,
                           z = (cz + n + (uint32_t)(o / 9) - 1u) % n;
            const uint32_t oc = x + n * (y + n * z);
            const uint32_t m = cntb[oc];
            for (uint32_t j = 0; j < m; ++j) {
                if (oc == c && j == i) continue;
                acc += 0.5 * pair_energy_full(a, recb[(size_t)oc * cap + j], R.scale, R.R2, lB, R.kappa, eps,
                                              ion_coupling);
            }
        }
        if (rec_is_ion(a.w) && ion_coupling && eps > 0.0) {
            for (uint32_t k = 0; k < R.ncores; ++k) {
                const uint4 cc = R.core_x[k];
                const int32_t dx = (int32_t)(cc.x - a.x), dy = (int32_t)(cc.y - a.y), dz = (int32_t)(cc.z - a.z);
                const double fx = dx * R.scale, fy = dy * R.scale, fz = dz * R.scale;
                const double rr = sqrt(fx * fx + fy * fy + fz * fz);
                const double sh = rr - R.core_delta[k];
                if (sh < 1.122462048309373) {
                    if (sh < 0.5) { acc += __longlong_as_double(0x7FF0000000000000ll); continue; }
                    const double ir2 = 1.0 / (sh * sh), ir6 = ir2 * ir2 * ir2;
                    acc += 4.0 * eps * (ir6 * ir6 - ir6) + eps;
                }
            }
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x == 0) out[c] = acc;
}

__global__ void k_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[4];
    philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, w);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = w[k];
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
hipError_t launch_bin(const SweepArgs& a, hipStream_t s)
{
    const uint32_t per = BIN_THREADS / 64;
    hipLaunchKernelGGL(k_bin, dim3((a.ncell_total + per - 1) / per), dim3(BIN_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename Real>
static hipError_t launch_phase_t(const SweepArgs& a, size_t lds, hipStream_t s)
{
    switch (a.phase_threads) {
    case 64: hipLaunchKernelGGL((k_phase<Real, 64>), dim3(a.ndom_total), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((k_phase<Real, 128>), dim3(a.ndom_total), dim3(128), lds, s, a); break;
    case 512: hipLaunchKernelGGL((k_phase<Real, 512>), dim3(a.ndom_total), dim3(512), lds, s, a); break;
    default: hipLaunchKernelGGL((k_phase<Real, 256>), dim3(a.ndom_total), dim3(256), lds, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_phase(const SweepArgs& a, size_t lds, hipStream_t s)
{
    return a.precision == 64 ? launch_phase_t<double>(a, lds, s) : launch_phase_t<float>(a, lds, s);
}

hipError_t launch_sweep_end(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy(const Replica* rep_dev, const Replica& rep_host, double lB, double eps, int ion_coupling,
                         int buf, double* out_per_cell, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(rep_host.ncells), dim3(64), 0, s, rep_dev, buf, lB, eps, ion_coupling,
                       out_per_cell);
    return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3((uint32_t)blocks), dim3(256), 0, s, n, ctr, k0, k1, out);
    return hipGetLastError();
}

hipError_t set_phase_lds_limit(size_t bytes)
{
    const void* fns[] = {(const void*)k_phase<float, 64>, (const void*)k_phase<float, 128>,
                         (const void*)k_phase<float, 256>, (const void*)k_phase<float, 512>,
                         (const void*)k_phase<double, 64>, (const void*)k_phase<double, 128>,
                         (const void*)k_phase<double, 256>, (const void*)k_phase<double, 512>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace crmc
